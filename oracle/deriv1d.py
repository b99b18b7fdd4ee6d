"""Oracle: derivative (d1, d2) loss rows of the 1D profile problems (FP64,
numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Methods, "Training Loss".  Besides the d0 loss on the residual, the
paper adds losses on its first and second derivatives, each on its own point
batch, L_d1 = 1/(N_d1 N_E d) sum rho sum_k sum_i (d_i R_k)^2 and
L_d2 = 1/(N_d2 N_E d^2) sum rho sum_k sum_ij (d_i d_j R_k)^2.  In 1D (d = 1,
N_E = 1) the rows are r = sqrt(c rho / N_d) d^n R / dy^n (c the loss weight).

For the 1D residual R = -lam Theta + V Theta', V = (1+lam) y + U:
  R'  = (1 + U') Theta' + V Theta'',
  R'' = U'' Theta' + (2 + lam + 2 U') Theta'' + V Theta''',
with U = H Theta (CCF) or U = Theta (local Burgers variant).  The Hilbert
transform commutes with d/dy, so U' = H[Theta'] and U'' = H[Theta''].
Theta is even for CCF, so Theta' is odd and Theta'' even.  On the half line:
  even f:  (H f)(y) = (1/pi) int_0^inf (f(t) - f(y)) 2y / (y^2 - t^2) dt,
  odd f:   (H f)(y) = (1/pi) int_0^inf (t f(t) - y f(y)) 2 / (y^2 - t^2) dt;
the odd form combines the two half lines into 2t / (y^2 - t^2) and subtracts
y f(y) times p.v. int_0^inf 2 / (y^2 - t^2) dt = 0.  Both use the d0 rows'
nodes t_j and weights w_j (Q_ij = w_j 2 y_i / (y_i^2 - t_j^2),
Q1_ij = w_j 2 / (y_i^2 - t_j^2)).

Derivatives in y are taken by truncated Taylor arithmetic (coefficients
f_k = f^(k)/k!, order 3): products by the Cauchy rule, powers and tanh by
their standard recurrences (Griewank and Walther, "Evaluating Derivatives",
chapter 13), through the whole composition y -> q(y) -> network -> envelope.
Everything is generic in the numpy dtype, so the parameter Jacobian is the
complex-step derivative.
"""
from __future__ import annotations

import numpy as np

from . import profile1d as p1

K = 3  # highest derivative order carried


# ------------------------------------------------------------ Taylor arithmetic
def tvar(y):
    """Taylor coefficients of the identity at y."""
    y = np.asarray(y)
    out = np.zeros((K + 1,) + y.shape, dtype=y.dtype)
    out[0] = y
    out[1] = 1.0
    return out


def tmul(a, b):
    out = np.zeros(np.broadcast_shapes(a.shape, b.shape), dtype=np.result_type(a, b))
    for k in range(K + 1):
        for j in range(k + 1):
            out[k] = out[k] + a[j] * b[k - j]
    return out


def tpow(a, p):
    """a^p for a with a_0 > 0: k a_0 u_k = sum_{j=1..k} (p j - (k - j)) a_j u_{k-j}."""
    u = np.zeros_like(a)
    u[0] = a[0] ** p
    for k in range(1, K + 1):
        acc = 0.0
        for j in range(1, k + 1):
            acc = acc + (p * j - (k - j)) * a[j] * u[k - j]
        u[k] = acc / (k * a[0])
    return u


def ttanh(z):
    """t = tanh(z) from t' = (1 - t^2) z': k t_k = sum_{j=1..k} j z_j s_{k-j}, s = 1 - t^2."""
    t = np.zeros_like(z)
    s = np.zeros_like(z)
    t[0] = np.tanh(z[0])
    s[0] = 1.0 - t[0] * t[0]
    for k in range(1, K + 1):
        acc = 0.0
        for j in range(1, k + 1):
            acc = acc + j * z[j] * s[k - j]
        t[k] = acc / k
        sk = 0.0
        for l in range(k + 1):
            sk = sk + t[l] * t[k - l]
        s[k] = -sk
    return t


def derivatives(c):
    """f^(k) = k! f_k."""
    out = np.array(c, copy=True)
    f = 1.0
    for k in range(1, K + 1):
        f *= k
        out[k] = out[k] * f
    return out


# ------------------------------------------------------------ the field in y
def field_taylor(theta, widths, y, lam, equation):
    """Taylor coefficients (K+1, n) of Theta(y) = E(y) NN(q(y))."""
    Y = tvar(np.asarray(y, dtype=np.float64))
    w = tmul(Y, Y)
    w[0] = w[0] + 1.0                                   # 1 + y^2
    q = tpow(w, -1.0 / (2.0 * (1.0 + lam)))
    h = q[:, None, :]                                   # (K+1, width, n)
    layers = p1.unpack(theta, widths)
    for l, (W, b) in enumerate(layers):
        z = np.einsum("ij,kjn->kin", W, h)
        z[0] = z[0] + b[:, None]
        h = ttanh(z) if l < len(layers) - 1 else z
    NN = h[:, 0, :]
    e = lam / (2.0 * (1.0 + lam))
    if equation == p1.CCF:
        E = tmul(tmul(Y, Y), tpow(w, e - 1.0))          # y^2 (1+y^2)^(e-1)
    elif equation == p1.BURGERS:
        E = tmul(Y, tpow(w, e - 0.5))                   # y (1+y^2)^(e-1/2)
    else:
        raise ValueError(equation)
    return tmul(E, NN)


def field_derivs(theta, widths, y, lam, equation):
    """(Theta, Theta', Theta'', Theta''') at y, shape (4, n)."""
    return derivatives(field_taylor(theta, widths, y, lam, equation))


# ------------------------------------------------------------ Hilbert terms
def hilbert_odd(y, t, what, f_nodes, f_points):
    """(H f)(y_i) ~= sum_j Q1_ij (t_j f(t_j) - y_i f(y_i)) for odd f."""
    y = np.asarray(y, dtype=np.float64)
    Q1 = what[None, :] * 2.0 / ((y[:, None] - t[None, :]) * (y[:, None] + t[None, :]))
    return (Q1 * (t[None, :] * f_nodes[None, :] - y[:, None] * f_points[:, None])).sum(axis=1)


def transform_derivs(prob, theta, y, F):
    """(U, U', U'') at y given the field derivatives F there (rows 0..2)."""
    if prob.equation == p1.BURGERS:
        return F[0], F[1], F[2]
    Ft = field_derivs(theta, prob.widths, prob.t, prob.lam, prob.equation)
    Q = p1.hilbert_matrix(y, prob.t, prob.what)
    U = p1.hilbert_even(Q, Ft[0], F[0])
    U1 = hilbert_odd(y, prob.t, prob.what, Ft[1], F[1])
    U2 = p1.hilbert_even(Q, Ft[2], F[2])
    return U, U1, U2


def residual_derivs(lam, y, F, U, U1, U2):
    """(R', R'') from the field derivatives F (Theta..Theta''') and U, U', U''."""
    V = (1.0 + lam) * y + U
    R1 = (1.0 + U1) * F[1] + V * F[2]
    R2 = U2 * F[1] + (2.0 + lam + 2.0 * U1) * F[2] + V * F[3]
    return R1, R2


def deriv_residuals(prob, theta, s1, s2):
    """Raw R' at the d1 points (mapped coordinates s1) and R'' at the d2 points s2."""
    out = []
    for order, s in ((1, s1), (2, s2)):
        if s is None or len(s) == 0:
            out.append(np.zeros(0, dtype=np.result_type(theta, np.float64)))
            continue
        _, y = p1.coords(np.asarray(s, dtype=np.float64), prob.lam)
        F = field_derivs(theta, prob.widths, y, prob.lam, prob.equation)
        U, U1, U2 = transform_derivs(prob, theta, y, F)
        R1, R2 = residual_derivs(prob.lam, y, F, U, U1, U2)
        out.append(R1 if order == 1 else R2)
    return out[0], out[1]


# ------------------------------------------------------------ rows and Jacobian
class Problem(p1.Problem):
    """A 1D problem with d1 rows (points s1, weight c_d1) and d2 rows (points
    s2, weight c_d2).  Row order: d0 rows, d1 rows, d2 rows, normalisation."""

    def __init__(self, base: p1.Problem, s1=None, s2=None, c_d1=1.0, c_d2=1.0):
        self.__dict__.update(base.__dict__)
        self.s1 = np.zeros(0) if s1 is None else np.asarray(s1, dtype=np.float64)
        self.s2 = np.zeros(0) if s2 is None else np.asarray(s2, dtype=np.float64)
        self.c_d1, self.c_d2 = float(c_d1), float(c_d2)
        self.n1, self.n2 = self.s1.size, self.s2.size
        self.m = self.n + self.n1 + self.n2 + 1

    def residual_rows(self, theta):
        R, _ = p1.raw_residual(self, theta)
        sc = np.sqrt(self.rho / self.n)
        R1, R2 = deriv_residuals(self, theta, self.s1, self.s2)
        r1 = np.sqrt(self.c_d1 / max(self.n1, 1)) * R1
        r2 = np.sqrt(self.c_d2 / max(self.n2, 1)) * R2
        NN1, _, _ = p1.mlp_jets(theta, self.widths, np.ones(1))
        rn = np.sqrt(self.c_norm) * (NN1[0] - self.c_target)
        return np.concatenate([sc * (R - self.f), r1, r2, [rn]])

    def jacobian(self, theta, h=1e-30):
        """Complex-step derivative over every parameter (no subtraction error)."""
        theta = np.asarray(theta, dtype=np.float64)
        out = np.empty((self.m, theta.size))
        for k in range(theta.size):
            tc = theta.astype(np.complex128)
            tc[k] += 1j * h
            out[:, k] = np.imag(self.residual_rows(tc)) / h
        return out


# ------------------------------------------------------------ lambda inference
def lambda_estimate(prob, theta):
    """Blow-up rate implied at the origin (Methods, "Identifying Admissible
    lambda Values", lambda inference: derivatives of the self-similar
    equation at the origin must vanish, which ties lambda to field values
    there).  For the even CCF profile R'(0) = 0 identically; with
    Theta = a y^2 + ..., U = c y + ..., R''(0) = 2a (2 + lam + 2c), so an exact
    profile has U'(0) = -(1 + lam/2):
    lam_hat = -2 (1 + U'(0)), with U'(0) = H[Theta'](0) by the odd half-line
    form at y = 0, -(2/pi) int_0^inf Theta'(t) / t dt, on the problem's nodes."""
    if prob.equation != p1.CCF:
        raise ValueError("lambda inference is defined for the CCF problem")
    Ft = field_derivs(theta, prob.widths, prob.t, prob.lam, prob.equation)
    U1_0 = hilbert_odd(np.zeros(1), prob.t, prob.what, Ft[1], np.zeros(1))[0]
    return -2.0 * (1.0 + U1_0), U1_0
