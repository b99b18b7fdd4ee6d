"""Oracle for the 2D self-similar profile stand-ins: coordinates, network jets
in y up to second order, fields, residual rows, parameter Jacobian (FP64,
numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed (arXiv 2509.14185, Methods):
- "Solution Modeling and Equation Factorisation": compactified coordinates
  z = (q, beta), q = (1+|y|^2)^{-1/(2(1+lambda))}, beta = y2/sqrt(1+|y|^2),
  passed to a tanh MLP; each field is a symmetry prefactor times the network
  output times a decay factor, e.g. Omega = (y1/sqrt(1+|y|^2)) NN q.
- "Training Loss": equation rows weighted by 1/(N N_E), derivative (d1)
  rows by 1/(N1 N_E d), a normalisation (data) row.
- "Validation Metrics for Solutions": max |R| over a validation grid.

Readings (the IPM and Boussinesq residuals are defined in the unpublished
supplementary material; these are stand-ins with the same structure):
- Points: s in [0,1)^2 mapped per axis to y_k = s_k / (1 - s_k) (quadrant).
- IPM-style (one field): Phi = (y1/rho) NN q, rho = sqrt(1+|y|^2);
  R = Phi + ((1+lam) y + (Phi, 0)) . grad Phi; d1 rows dR/dy1, dR/dy2 on a
  second point set; symmetry rows dPhi/dy2 (y1, 0) = 0 on y2 = 0.
- Boussinesq-type (three fields Omega, Theta, Psi from one 3-output MLP):
  Omega = (y1/rho) NN_0 q, Theta = NN_1 q, Psi = (y1/rho) NN_2 q rho^2;
  with U = (-Psi_2, Psi_1):
  R_Omega = Omega + ((1+lam) y + U) . grad Omega - Theta_1,
  R_Theta = (1-lam) Theta + ((1+lam) y + U) . grad Theta,
  R_Psi = Psi_11 + Psi_22 - Omega; boundary rows Psi(y1, 0) = 0.
- Normalisation row sqrt(c_norm) (NN_0(q=1, beta=0) - c_target) (the origin).
- Row order: equation rows point by point (fields interleaved per point),
  then d1 rows (dR/dy1, dR/dy2 per point), then the y2 = 0 rows, then the
  normalisation row.  Weights rho = 1.

Jets: arrays with a leading axis of 6 components (f, f_1, f_2, f_11, f_12,
f_22) of derivatives with respect to y, composed by the product and chain
rules (Taylor mode).  Everything is written for generic numpy dtypes so the
parameter Jacobian can be taken by the complex-step derivative, which has no
subtraction error: dr/dtheta_k = Im r(theta + i h e_k) / h.

Parameter layout: per affine layer, W row-major (w_out x w_in) then b.
"""
from __future__ import annotations

import numpy as np

NC = 6  # f, f_1, f_2, f_11, f_12, f_22
IPM2D, BOUSS2D = "ipm2d", "bouss2d"


# ---------------------------------------------------------------- jets (order 2)
def jvar(y, a):
    """Jet of the coordinate y_a (a = 1 or 2)."""
    out = np.zeros((NC,) + np.shape(y), dtype=np.asarray(y).dtype)
    out[0] = y
    out[a] = 1.0
    return out


def jconst(c, like):
    out = np.zeros_like(like)
    out[0] = c
    return out


def jmul(f, g):
    """Product rule up to second order."""
    out = np.empty(np.broadcast_shapes(f.shape, g.shape), dtype=np.result_type(f, g))
    out[0] = f[0] * g[0]
    out[1] = f[1] * g[0] + f[0] * g[1]
    out[2] = f[2] * g[0] + f[0] * g[2]
    out[3] = f[3] * g[0] + 2.0 * f[1] * g[1] + f[0] * g[3]
    out[4] = f[4] * g[0] + f[1] * g[2] + f[2] * g[1] + f[0] * g[4]
    out[5] = f[5] * g[0] + 2.0 * f[2] * g[2] + f[0] * g[5]
    return out


def jchain(f, v, d1, d2):
    """phi(f) given phi(f0) = v, phi'(f0) = d1, phi''(f0) = d2 (chain rule)."""
    out = np.empty(f.shape, dtype=np.result_type(f, v, d1, d2))
    out[0] = v
    out[1] = d1 * f[1]
    out[2] = d1 * f[2]
    out[3] = d2 * f[1] * f[1] + d1 * f[3]
    out[4] = d2 * f[1] * f[2] + d1 * f[4]
    out[5] = d2 * f[2] * f[2] + d1 * f[5]
    return out


def jtanh(f):
    t = np.tanh(f[0])
    s = 1.0 - t * t
    return jchain(f, t, s, -2.0 * t * s)


def jpow(f, m):
    """f^m for f > 0 (real exponent)."""
    x = f[0]
    return jchain(f, x ** m, m * x ** (m - 1.0), m * (m - 1.0) * x ** (m - 2.0))


# ---------------------------------------------------------------- geometry
def coords(s):
    """Per-axis map of s in [0,1) to y in [0, inf)."""
    s = np.asarray(s)
    return s / (1.0 - s)


def base_jets(y1, y2):
    """Jets of y1, y2 and u = 1 + |y|^2."""
    Y1 = jvar(np.asarray(y1, dtype=np.float64), 1)
    Y2 = jvar(np.asarray(y2, dtype=np.float64), 2)
    U = jmul(Y1, Y1) + jmul(Y2, Y2)
    U[0] += 1.0
    return Y1, Y2, U


def net_inputs(y1, y2, lam):
    """Jets of the network inputs q and beta."""
    Y1, Y2, U = base_jets(y1, y2)
    q = jpow(U, -1.0 / (2.0 * (1.0 + lam)))
    beta = jmul(Y2, jpow(U, -0.5))
    return q, beta


def envelopes(y1, y2, lam, equation):
    """Jets of the per-field factors multiplying the network outputs."""
    Y1, Y2, U = base_jets(y1, y2)
    q = jpow(U, -1.0 / (2.0 * (1.0 + lam)))
    odd = jmul(Y1, jpow(U, -0.5))  # y1 / rho
    if equation == IPM2D:
        return [jmul(odd, q)]
    if equation == BOUSS2D:
        return [jmul(odd, q), q, jmul(jmul(odd, q), U)]
    raise ValueError(equation)


# ---------------------------------------------------------------- network
def unpack(theta, widths):
    layers, o = [], 0
    for a, b in zip(widths[:-1], widths[1:]):
        W = theta[o:o + a * b].reshape(b, a)
        o += a * b
        bias = theta[o:o + b]
        o += b
        layers.append((W, bias))
    assert o == len(theta)
    return layers


def mlp_jets(theta, widths, y1, y2, lam):
    """NN output jets at the points: shape (6, n_out, npts)."""
    q, beta = net_inputs(y1, y2, lam)
    h = np.stack([q, beta], axis=1)  # (6, 2, npts)
    layers = unpack(theta, widths)
    for li, (W, b) in enumerate(layers):
        z = np.einsum("kj,cjp->ckp", W, h)
        z[0] = z[0] + b[:, None]
        h = z if li == len(layers) - 1 else jtanh(z)
    return h


def fields(theta, widths, y1, y2, lam, equation):
    """Field jets, list of (6, npts) arrays."""
    nn = mlp_jets(theta, widths, y1, y2, lam)
    return [jmul(E, nn[:, f]) for f, E in enumerate(envelopes(y1, y2, lam, equation))]


# ---------------------------------------------------------------- residuals
def _mul1(a, b):
    """Product rule for first-order jets (value, d1, d2) along axis 0."""
    return np.stack([a[0] * b[0], a[1] * b[0] + a[0] * b[1], a[2] * b[0] + a[0] * b[2]])


def ipm_residual(Phi, y1, y2, lam):
    """R = Phi + ((1+lam) y1 + Phi) Phi_1 + (1+lam) y2 Phi_2."""
    return Phi[0] + ((1.0 + lam) * y1 + Phi[0]) * Phi[1] + (1.0 + lam) * y2 * Phi[2]


def ipm_residual_d1(Phi, y1, y2, lam):
    """(dR/dy1, dR/dy2) by first-order jets of every factor of R."""
    one = np.ones_like(Phi[0])
    zero = np.zeros_like(Phi[0])
    F = Phi[[0, 1, 2]]
    G1 = Phi[[1, 3, 4]]  # Phi_1 and its derivatives
    G2 = Phi[[2, 4, 5]]
    V1 = np.stack([(1.0 + lam) * y1 + Phi[0], (1.0 + lam) * one + Phi[1], Phi[2]])
    V2 = np.stack([(1.0 + lam) * y2 * one, zero, (1.0 + lam) * one])
    R = F + _mul1(V1, G1) + _mul1(V2, G2)
    return R[1], R[2]


def bouss_residuals(Om, Th, Ps, y1, y2, lam):
    V1 = (1.0 + lam) * y1 - Ps[2]
    V2 = (1.0 + lam) * y2 + Ps[1]
    Ro = Om[0] + V1 * Om[1] + V2 * Om[2] - Th[1]
    Rt = (1.0 - lam) * Th[0] + V1 * Th[1] + V2 * Th[2]
    Rp = Ps[3] + Ps[5] - Om[0]
    return Ro, Rt, Rp


# ---------------------------------------------------------------- problem
class Problem:
    """One 2D profile problem; s, s1: (n,2), (n1,2); se: (ne,) on y2 = 0."""

    def __init__(self, equation, widths, lam, s, s1, se, sval, c_norm=1.0, c_target=1.0):
        self.equation = equation
        self.widths = list(widths)
        self.lam = float(lam)
        self.P = int(sum(b * (a + 1) for a, b in zip(widths[:-1], widths[1:])))
        y = coords(np.asarray(s, dtype=np.float64).reshape(-1, 2))
        self.y1, self.y2 = y[:, 0].copy(), y[:, 1].copy()
        y = coords(np.asarray(s1, dtype=np.float64).reshape(-1, 2))
        self.d1y1, self.d1y2 = y[:, 0].copy(), y[:, 1].copy()
        self.ey1 = coords(np.asarray(se, dtype=np.float64))
        self.ey2 = np.zeros_like(self.ey1)
        y = coords(np.asarray(sval, dtype=np.float64).reshape(-1, 2))
        self.vy1, self.vy2 = y[:, 0].copy(), y[:, 1].copy()
        self.c_norm, self.c_target = float(c_norm), float(c_target)
        self.n, self.n1, self.ne = len(self.y1), len(self.d1y1), len(self.ey1)
        self.n_eq = 1 if equation == IPM2D else 3
        if equation == BOUSS2D and self.n1:
            raise ValueError("d1 rows are defined for the IPM-style problem")

    @classmethod
    def from_inputs(cls, inp):
        return cls(inp["equation"], inp["widths"], inp["lam"], inp["s"], inp["s1"], inp["se"], inp["sval"],
                   inp["c_norm"], inp["c_target"])

    @property
    def m(self):
        return self.n * self.n_eq + 2 * self.n1 + self.ne + 1

    def raw(self, theta, y1, y2):
        """Raw residuals at points: list of n_eq arrays."""
        F = fields(theta, self.widths, y1, y2, self.lam, self.equation)
        if self.equation == IPM2D:
            return [ipm_residual(F[0], y1, y2, self.lam)]
        return list(bouss_residuals(F[0], F[1], F[2], y1, y2, self.lam))

    def row_map(self, rows):
        """(kind, point, component) of each global row index; kind 0 equation
        rows (component = equation), 1 d1 rows (component = direction), 2 the
        y2 = 0 rows, 3 the normalisation row."""
        rows = np.asarray(rows)
        ne0 = self.n * self.n_eq
        n10 = ne0 + 2 * self.n1
        nb0 = n10 + self.ne
        kind = np.where(rows < ne0, 0, np.where(rows < n10, 1, np.where(rows < nb0, 2, 3)))
        pt = np.where(kind == 0, rows // self.n_eq,
                      np.where(kind == 1, (rows - ne0) // 2, np.where(kind == 2, rows - n10, 0)))
        comp = np.where(kind == 0, rows % self.n_eq, np.where(kind == 1, (rows - ne0) % 2, 0))
        return kind, pt, comp

    def residual_rows(self, theta, rows=None):
        """Scaled residual rows (all, or the listed global row indices)."""
        if rows is None:
            rows = np.arange(self.m)
        kind, pt, comp = self.row_map(rows)
        lam = self.lam
        out = np.zeros(len(rows), dtype=np.result_type(theta, np.float64))
        sel = kind == 0
        if sel.any():
            R = self.raw(theta, self.y1[pt[sel]], self.y2[pt[sel]])
            v = np.stack(R, axis=0)[comp[sel], np.arange(sel.sum())]
            out[sel] = np.sqrt(1.0 / (self.n * self.n_eq)) * v
        sel = kind == 1
        if sel.any():
            a, b = self.d1y1[pt[sel]], self.d1y2[pt[sel]]
            F = fields(theta, self.widths, a, b, lam, self.equation)
            d = np.stack(ipm_residual_d1(F[0], a, b, lam), axis=0)[comp[sel], np.arange(sel.sum())]
            out[sel] = np.sqrt(1.0 / (2.0 * self.n1)) * d
        sel = kind == 2
        if sel.any():
            a, b = self.ey1[pt[sel]], self.ey2[pt[sel]]
            F = fields(theta, self.widths, a, b, lam, self.equation)
            edge = F[0][2] if self.equation == IPM2D else F[2][0]
            out[sel] = np.sqrt(1.0 / self.ne) * edge
        sel = kind == 3
        if sel.any():
            nn0 = mlp_jets(theta, self.widths, np.zeros(1), np.zeros(1), lam)[0, 0, 0]
            out[sel] = np.sqrt(self.c_norm) * (nn0 - self.c_target)
        return out

    def jacobian(self, theta, rows=None, cols=None, h=1e-30):
        """dr/dtheta by the complex-step derivative, one column at a time
        (all rows, or the listed ones)."""
        theta = np.asarray(theta, dtype=np.float64)
        cols = np.arange(self.P) if cols is None else np.asarray(cols)
        nrow = self.m if rows is None else len(rows)
        J = np.empty((nrow, len(cols)))
        for k, col in enumerate(cols):
            t = theta.astype(np.complex128)
            t[col] += 1j * h
            J[:, k] = self.residual_rows(t, rows).imag / h
        return J

    def validation_max(self, theta):
        return float(max(np.max(np.abs(R)) for R in self.raw(theta, self.vy1, self.vy2)))

    def train_max(self, theta):
        return float(max(np.max(np.abs(R)) for R in self.raw(theta, self.y1, self.y2)))
