"""Oracle: second stage of multi-stage training for the 1D profile problems
(FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper: Methods, "Multi-stage Training".  The solution is written as
Theta = Theta_1 + eps Theta_2 with a trained first stage Theta_1 and a small
eps; substituted into the equation this gives, to first order in eps, the
linear equation -eps D[Theta_1] Theta_2 = R[Theta_1] for the second stage,
D the linearisation of the residual around Theta_1.  The second network is
a Fourier feature network: a layer [cos(B x), sin(B x)] with fixed Gaussian
weights B ~ N(0, sigma), sigma = 2 pi f_d (f_d the dominant frequency of the
first-stage residual), feeds a tanh MLP.

For R = -lam Theta + ((1+lam) y + U) Theta' (U = H Theta, CCF; U = Theta for
the local variant):
  D[Theta_1] Phi = -lam Phi + V_1 Phi' + U[Phi] Theta_1',
V_1 = (1+lam) y + U_1.  Because R is quadratic in Theta,
R[Theta_1 + eps Phi] = R[Theta_1] + eps D[Theta_1] Phi + eps^2 U[Phi] Phi'
exactly.

Readings (not fixed by the paper): the Fourier layer acts on the network
input q directly, features cos(b_k q), sin(b_k q), k = 1..F (a first linear
layer with fixed weights folds into b); the stage-2 field carries the same
envelope, Theta_2 = E(y) NN_2(q(y)); the stage-2 rows are
r_i = sqrt(rho_i / N) (R_1,i + eps D_i) and the normalisation row
sqrt(c_norm) NN_2(q = 1) (the combined field keeps NN(1) = 1); eps is an
input.
"""
from __future__ import annotations

import numpy as np

from . import profile1d as p1


def fourier_features(x, b):
    """phi = [cos(b x), sin(b x)] and d phi / dx, shapes (2F, n)."""
    x = np.asarray(x)
    u = b[:, None] * x[None, :]
    c, s = np.cos(u), np.sin(u)
    return np.concatenate([c, s]), np.concatenate([-b[:, None] * s, b[:, None] * c])


def fourier_mlp_jets(theta, widths, b, x):
    """NN and dNN/dx of the tanh MLP (widths[0] = 2F) applied to the Fourier
    features of x: z^1 = W^1 phi + b^1, z^1_x = W^1 phi_x, then as mlp_jets."""
    layers = p1.unpack(theta, widths)
    h, hx = fourier_features(x, b)
    for l, (W, bb) in enumerate(layers):
        z = W @ h + bb[:, None]
        zx = W @ hx
        if l < len(layers) - 1:
            t = np.tanh(z)
            h, hx = t, (1.0 - t * t) * zx
        else:
            h, hx = z, zx
    return h[0], hx[0]


class Stage2Problem:
    """Second-stage rows around a fixed first stage (theta1 on problem base)."""

    def __init__(self, base: p1.Problem, theta1, widths2, b, eps):
        self.base = base
        self.widths = list(widths2)
        self.b = np.asarray(b, dtype=np.float64)
        assert self.widths[0] == 2 * self.b.size
        self.eps = float(eps)
        self.lam = base.lam
        self.n = base.n
        self.P = sum(w * (a + 1) for a, w in zip(self.widths[:-1], self.widths[1:]))
        self.m = self.n + 1
        R1, aux = p1.raw_residual(base, theta1)
        self.R1 = R1
        self.T1y = aux["Thy"]
        self.V1 = (1.0 + base.lam) * base.y + aux["U"]
        self.theta1 = np.asarray(theta1, dtype=np.float64)

    def field2(self, theta2, y):
        q = p1.q_of_y(y, self.lam)
        NN, NNq = fourier_mlp_jets(theta2, self.widths, self.b, q)
        E, Ey = p1.envelope(y, self.lam, self.base.equation)
        return E * NN, Ey * NN + E * p1.dq_dy(y, self.lam) * NNq

    def linearised(self, theta2):
        """D[Theta_1] Theta_2 at the collocation points."""
        base = self.base
        T2, T2y = self.field2(theta2, base.y)
        if base.equation == p1.CCF:
            Tt, _ = self.field2(theta2, base.t)
            U2 = p1.hilbert_even(base.Q, Tt, T2)
        else:
            U2 = T2
        return -self.lam * T2 + self.V1 * T2y + U2 * self.T1y

    def residual_rows(self, theta2):
        sc = np.sqrt(self.base.rho / self.n)
        r = sc * (self.R1 + self.eps * self.linearised(theta2))
        NN1, _ = fourier_mlp_jets(theta2, self.widths, self.b, np.ones(1))
        return np.concatenate([r, [np.sqrt(self.base.c_norm) * NN1[0]]])

    def jacobian(self, theta2, h=1e-30):
        """Complex-step derivative over every parameter."""
        theta2 = np.asarray(theta2, dtype=np.float64)
        out = np.empty((self.m, theta2.size))
        for k in range(theta2.size):
            tc = theta2.astype(np.complex128)
            tc[k] += 1j * h
            out[:, k] = np.imag(self.residual_rows(tc)) / h
        return out
