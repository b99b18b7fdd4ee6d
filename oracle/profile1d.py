"""Oracle for the 1D self-similar profile problem: geometry, network jets,
envelope, residual rows, parameter Jacobian (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed (arXiv 2509.14185, Methods):
- "Self-similar Solutions": phi(x,t) = (1-t)^{k(lambda)} Phi(y),
  y = (1-t)^{-(1+lambda)} x, giving a static equation E(Phi, lambda) = 0.
- "Solution Modeling and Equation Factorisation": compactified coordinate
  q = (1+|y|^2)^{-1/(2(1+lambda))}; the network sees q; the field is an
  envelope (symmetry and far-field factor) times the network output; tanh
  MLP.
- "Training Loss": d0 rows weighted by rho / (N_d0 N_E); data (normalisation)
  row c_norm (Phi(y_norm) - C_norm)^2.
- "Validation Metrics for Solutions": max |R| over a validation grid.

Readings where the paper is silent (the supplementary material that defines
the CCF residual is not published):
- CCF equation theta_t + (H theta) theta_x = 0 with the self-similar ansatz
  (k = lambda) gives R = -lam*Theta + ((1+lam) y + H Theta) Theta_y.
  The velocity sign is u = +H theta.
- Theta is even, Theta(0) = 0; domain y >= 0.  Envelope
  E(y) = y^2/(1+y^2) * q^{-lam} (evenness, Theta ~ y^2 at 0, far-field growth
  |y|^{lam/(1+lam)}).  Normalisation NN(q=1) = 1.
- H Theta on the half line for even Theta, singularity subtracted:
  (H Theta)(y) = (1/pi) int_0^inf (Theta(t) - Theta(y)) 2y/(y^2 - t^2) dt,
  discretised with nodes t_j = y(s_j) and weights (ws_j dt/ds)/pi.
- Local "Burgers" variant (H Theta replaced by Theta), odd field with
  envelope y/sqrt(1+y^2) * q^{-lam}; it has closed-form profiles.
- Rows: r_i = sqrt(rho_i/N) (R_i - f_i) for i < N (f is an optional source),
  r_N = sqrt(c_norm) (NN(q=1) - c_target).  h = |r|^2/2.

Parameter layout: per affine layer, W row-major (w_out x w_in) then b.
All functions are written for generic numpy dtypes so that the complex-step
derivative can be taken through them.
"""
from __future__ import annotations

import numpy as np

CCF = "ccf1d"
BURGERS = "burgers1d"


# ----------------------------------------------------------------------------
# Geometry: mapped coordinate s in [0,1), q = 1 - s, y(q) from
# q = (1 + y^2)^(-1/(2(1+lam))).
# ----------------------------------------------------------------------------
def coords(s, lam):
    """Return (q, y) for mapped points s: q = 1 - s, y = sqrt(q^{-2(1+lam)} - 1)."""
    s = np.asarray(s)
    q = 1.0 - s
    y = np.sqrt(np.expm1(-2.0 * (1.0 + lam) * np.log1p(-s)))
    return q, y


def dy_ds(s, lam):
    """dy/ds; from y^2 = q^{-2(1+lam)} - 1: 2 y y' = 2 (1+lam) q^{-2(1+lam)-1}."""
    q, y = coords(s, lam)
    return (1.0 + lam) * q ** (-2.0 * (1.0 + lam) - 1.0) / y


def q_of_y(y, lam):
    return (1.0 + y * y) ** (-1.0 / (2.0 * (1.0 + lam)))


def dq_dy(y, lam):
    """d/dy (1+y^2)^(-1/(2(1+lam)))."""
    a = -1.0 / (2.0 * (1.0 + lam))
    return a * 2.0 * y * (1.0 + y * y) ** (a - 1.0)


def envelope(y, lam, equation):
    """(E, dE/dy).  q^{-lam} = (1+y^2)^{e} with e = lam/(2(1+lam))."""
    e = lam / (2.0 * (1.0 + lam))
    w = 1.0 + y * y
    if equation == CCF:
        # E = y^2/(1+y^2) * q^{-lam} = y^2 (1+y^2)^{e-1}
        E = y * y * w ** (e - 1.0)
        Ey = 2.0 * y * w ** (e - 1.0) + y * y * (e - 1.0) * 2.0 * y * w ** (e - 2.0)
    elif equation == BURGERS:
        # E = y/sqrt(1+y^2) * q^{-lam} = y (1+y^2)^{e-1/2}
        E = y * w ** (e - 0.5)
        Ey = w ** (e - 0.5) + y * (e - 0.5) * 2.0 * y * w ** (e - 1.5)
    else:
        raise ValueError(equation)
    return E, Ey


# ----------------------------------------------------------------------------
# tanh MLP with first input-derivative jet (scalar input x, scalar output).
# ----------------------------------------------------------------------------
def unpack(theta, widths):
    layers, o = [], 0
    for a, b in zip(widths[:-1], widths[1:]):
        W = theta[o:o + a * b].reshape(b, a)
        o += a * b
        bb = theta[o:o + b]
        o += b
        layers.append((W, bb))
    assert o == len(theta), "theta length does not match widths"
    return layers


def mlp_jets(theta, widths, x):
    """Forward pass with the input-derivative jet.

    z^l = W^l h^{l-1} + b^l, h^l = tanh(z^l) (hidden), linear output layer;
    z^l_x = W^l h^{l-1}_x, h^l_x = (1 - tanh(z^l)^2) z^l_x, h^0 = x, h^0_x = 1.
    Returns (NN, NN_x, cache) with cache = list of (h^{l-1}, h^{l-1}_x, z^l, z^l_x).
    Arrays are (width, n_points).
    """
    layers = unpack(theta, widths)
    x = np.asarray(x)
    h = x[None, :]
    hx = np.ones_like(h)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = W @ h + b[:, None]
        zx = W @ hx
        cache.append((h, hx, z, zx))
        if l < len(layers) - 1:
            t = np.tanh(z)
            h = t
            hx = (1.0 - t * t) * zx
        else:
            h, hx = z, zx
    return h[0], hx[0], cache


def mlp_param_rows(theta, widths, x, s0, s1):
    """Rows s0_i dNN(x_i)/dtheta + s1_i dNN_x(x_i)/dtheta, shape (n, P).

    Reverse sweep through the jet recurrence of mlp_jets:
      dL/dW^l = zbar^l (x) h^{l-1} + zbar_x^l (x) h_x^{l-1},  dL/db^l = zbar^l,
      hbar = W^T zbar, hbar_x = W^T zbar_x, and through h = tanh z,
      h_x = (1 - t^2) z_x:
      zbar_x^{l-1} = hbar_x (1-t^2),
      zbar^{l-1}   = hbar (1-t^2) - 2 t (1-t^2) z_x^{l-1} hbar_x.
    """
    layers = unpack(theta, widths)
    _, _, cache = mlp_jets(theta, widths, x)
    n = np.asarray(x).shape[0]
    zb = np.asarray(s0)[None, :] * np.ones((1, n))
    zbx = np.asarray(s1)[None, :] * np.ones((1, n))
    blocks = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h, hx, _, _ = cache[l]
        dW = zb.T[:, :, None] * h.T[:, None, :] + zbx.T[:, :, None] * hx.T[:, None, :]
        blocks.append(np.concatenate([dW.reshape(n, -1), zb.T], axis=1))
        if l > 0:
            hb = W.T @ zb
            hbx = W.T @ zbx
            _, _, zprev, zxprev = cache[l - 1]
            t = np.tanh(zprev)
            d = 1.0 - t * t
            zbx = hbx * d
            zb = hb * d - 2.0 * t * d * zxprev * hbx
    return np.concatenate(blocks[::-1], axis=1)


# ----------------------------------------------------------------------------
# Field, Hilbert term and residual.
# ----------------------------------------------------------------------------
def field(theta, widths, y, lam, equation):
    """Theta(y) = E(y) NN(q(y)) and Theta_y = E_y NN + E q_y NN_q."""
    q = q_of_y(y, lam)
    NN, NNq, _ = mlp_jets(theta, widths, q)
    E, Ey = envelope(y, lam, equation)
    qy = dq_dy(y, lam)
    return E * NN, Ey * NN + E * qy * NNq, (NN, NNq, E, Ey, qy)


def hilbert_weights(sq, wq, lam):
    """Nodes t_j = y(s_j) and weights (ws_j dt/ds(s_j)) / pi."""
    _, t = coords(sq, lam)
    return t, wq * dy_ds(sq, lam) / np.pi


def hilbert_matrix(y, t, what):
    """Q_ij = what_j * 2 y_i / ((y_i - t_j)(y_i + t_j))."""
    y = np.asarray(y, dtype=np.float64)
    return what[None, :] * 2.0 * y[:, None] / ((y[:, None] - t[None, :]) * (y[:, None] + t[None, :]))


def hilbert_even(Q, f_nodes, f_points):
    """(H f)(y_i) ~= sum_j Q_ij (f(t_j) - f(y_i)) for even f on the half line."""
    return (Q * (f_nodes[None, :] - f_points[:, None])).sum(axis=1)


def residual_operator(lam, y, Th, Thy, U):
    """R = -lam Theta + ((1+lam) y + U) Theta_y  (U = H Theta for CCF, Theta for Burgers)."""
    return -lam * Th + ((1.0 + lam) * y + U) * Thy


class Problem:
    """Bundle of the problem constants and point sets (all FP64 numpy)."""

    def __init__(self, equation, widths, lam, s, rho=None, f=None, sq=None, wq=None,
                 sval=None, c_norm=1.0, c_target=1.0):
        self.equation = equation
        self.widths = list(widths)
        self.lam = float(lam)
        self.s = np.asarray(s, dtype=np.float64)
        self.n = self.s.size
        self.rho = np.ones(self.n) if rho is None else np.asarray(rho, dtype=np.float64)
        self.f = np.zeros(self.n) if f is None else np.asarray(f, dtype=np.float64)
        self.c_norm = float(c_norm)
        self.c_target = float(c_target)
        _, self.y = coords(self.s, self.lam)
        self.sval = None if sval is None else np.asarray(sval, dtype=np.float64)
        if equation == CCF:
            self.t, self.what = hilbert_weights(np.asarray(sq), np.asarray(wq), self.lam)
            self.Q = hilbert_matrix(self.y, self.t, self.what)
        self.P = sum(b * (a + 1) for a, b in zip(self.widths[:-1], self.widths[1:]))
        self.m = self.n + 1

    @classmethod
    def from_inputs(cls, inp, equation=None):
        return cls(equation or inp["equation"], inp["widths"], inp["lam"], inp["s"], inp["rho"],
                   inp["f"], inp["sq"], inp["wq"], inp["sval"], inp["c_norm"], inp["c_target"])


def raw_residual(prob, theta, y=None, Q=None):
    """R at points y (default: the collocation points), and the pieces used for J."""
    if y is None:
        y, Q = prob.y, getattr(prob, "Q", None)
    Th, Thy, parts = field(theta, prob.widths, y, prob.lam, prob.equation)
    if prob.equation == CCF:
        if Q is None:
            Q = hilbert_matrix(y, prob.t, prob.what)
        Tt, _, _ = field(theta, prob.widths, prob.t, prob.lam, prob.equation)
        U = hilbert_even(Q, Tt, Th)
    else:
        U = Th
    R = residual_operator(prob.lam, y, Th, Thy, U)
    return R, dict(Th=Th, Thy=Thy, U=U, parts=parts)


def residual_rows(prob, theta):
    """r (length m = N + 1): scaled collocation rows, then the data row."""
    R, _ = raw_residual(prob, theta)
    sc = np.sqrt(prob.rho / prob.n)
    NN1, _, _ = mlp_jets(theta, prob.widths, np.ones(1))
    rn = np.sqrt(prob.c_norm) * (NN1[0] - prob.c_target)
    return np.concatenate([sc * (R - prob.f), [rn]])


def jacobian(prob, theta, rows=None):
    """J = dr/dtheta (m x P), or only the listed rows.

    Collocation row i (scale sc_i = sqrt(rho_i/N)):
      CCF:  dR_i = (-lam E_i + V_i E_y,i - Theta_y,i c_i E_i) dNN_i
                  + V_i E_i q_y,i dNN_q,i + Theta_y,i sum_j Q_ij B_j,
            V = (1+lam) y + U, c_i = sum_j Q_ij, B_j = d Theta(t_j)/dtheta.
      Burgers: R = -lam U + ((1+lam) y + U) U_y with U = Theta:
            dR_i = ((Theta_y - lam) E + ((1+lam) y + Theta) E_y) dNN
                  + ((1+lam) y + Theta) E q_y dNN_q.
    Data row: sqrt(c_norm) dNN(q=1).
    """
    lam = prob.lam
    R, aux = raw_residual(prob, theta)
    Th, Thy, U = aux["Th"], aux["Thy"], aux["U"]
    NN, NNq, E, Ey, qy = aux["parts"]
    sc = np.sqrt(prob.rho / prob.n)
    y = prob.y
    if rows is None:
        rows = np.arange(prob.m)
    rows = np.asarray(rows)
    coll = rows[rows < prob.n]
    out = np.zeros((rows.size, prob.P))
    if coll.size:
        if prob.equation == CCF:
            V = (1.0 + lam) * y + U
            c = prob.Q.sum(axis=1)
            s0 = -lam * E + V * Ey - Thy * c * E
            s1 = V * E * qy
        else:
            V = (1.0 + lam) * y + Th
            s0 = (Thy - lam) * E + V * Ey
            s1 = V * E * qy
        q = q_of_y(y[coll], lam)
        loc = mlp_param_rows(theta, prob.widths, q, s0[coll], s1[coll])
        if prob.equation == CCF:
            tq = q_of_y(prob.t, lam)
            Et, _ = envelope(prob.t, lam, prob.equation)
            B = mlp_param_rows(theta, prob.widths, tq, Et, np.zeros_like(Et))
            loc = loc + Thy[coll][:, None] * (prob.Q[coll] @ B)
        out[rows < prob.n] = sc[coll][:, None] * loc
    if np.any(rows == prob.n):
        d = mlp_param_rows(theta, prob.widths, np.ones(1), np.ones(1), np.zeros(1))
        out[rows == prob.n] = np.sqrt(prob.c_norm) * d[0]
    return out


def validation_max(prob, theta):
    """max |R| over the validation grid (raw, unscaled residual)."""
    _, yv = coords(prob.sval, prob.lam)
    R, _ = raw_residual(prob, theta, y=yv)
    return float(np.max(np.abs(R)))
