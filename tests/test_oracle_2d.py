"""Pins of the 2D oracle (oracle/profile2d.py) against independent references:
sympy symbolic derivatives of the same fields and residuals written as plain
expressions in y (jets, envelopes, residuals, d1 and boundary rows), central
finite differences and sympy parameter derivatives for the complex-step
Jacobian, and closed forms of the coordinate map."""
import numpy as np
import pytest
import sympy as sp

import workloads
from oracle import gn as ogn
from oracle import profile2d as p2

Y1, Y2 = sp.symbols("y1 y2", real=True)
COMPS = [(), (Y1,), (Y2,), (Y1, Y1), (Y1, Y2), (Y2, Y2)]


def sym_net(theta, widths, lam):
    """sympy expressions of the network outputs as functions of (y1, y2)."""
    u = 1 + Y1 ** 2 + Y2 ** 2
    h = [u ** (-1 / (2 * (1 + lam))), Y2 / sp.sqrt(u)]
    o = 0
    for li, (a, b) in enumerate(zip(widths[:-1], widths[1:])):
        W = theta[o:o + a * b].reshape(b, a)
        o += a * b
        bias = theta[o:o + b]
        o += b
        z = [sum(float(W[k, j]) * h[j] for j in range(a)) + float(bias[k]) for k in range(b)]
        h = z if li == len(widths) - 2 else [sp.tanh(v) for v in z]
    return h


def sym_fields(theta, widths, lam, equation):
    u = 1 + Y1 ** 2 + Y2 ** 2
    q = u ** (-1 / (2 * (1 + lam)))
    odd = Y1 / sp.sqrt(u)
    nn = sym_net(theta, widths, lam)
    if equation == p2.IPM2D:
        return [odd * q * nn[0]]
    return [odd * q * nn[0], q * nn[1], odd * q * u * nn[2]]


def evaluate(expr, pts):
    f = sp.lambdify((Y1, Y2), expr, "numpy")
    return np.array([float(f(a, b)) for a, b in pts])


def jets_of(expr, pts):
    return np.stack([evaluate(sp.diff(expr, *c) if c else expr, pts) for c in COMPS])


PTS = [(0.3, 0.7), (1.7, 0.2), (0.05, 2.5), (4.0, 3.0)]


@pytest.fixture(scope="module")
def tiny():
    widths = [2, 3, 2, 3]
    theta = np.random.default_rng(5).uniform(-0.8, 0.8, sum(b * (a + 1) for a, b in zip(widths[:-1], widths[1:])))
    return widths, theta


def test_coordinate_map_closed_forms():
    s = np.array([0.0, 0.5, 0.75])
    assert np.allclose(p2.coords(s), [0.0, 1.0, 3.0], rtol=0, atol=0)
    q, beta = p2.net_inputs(np.array([0.0, 3.0]), np.array([0.0, 4.0]), 1.0)
    # |y| = 5: q = 26^{-1/4}, beta = 4/sqrt(26); at the origin q = 1, beta = 0
    assert q[0, 0] == 1.0 and beta[0, 0] == 0.0
    assert abs(q[0, 1] - 26.0 ** -0.25) < 1e-15 and abs(beta[0, 1] - 4.0 / np.sqrt(26.0)) < 1e-15


def test_network_jets_match_sympy(tiny):
    widths, theta = tiny
    lam = 0.4721
    y1 = np.array([p[0] for p in PTS])
    y2 = np.array([p[1] for p in PTS])
    got = p2.mlp_jets(theta, widths, y1, y2, lam)
    for k, e in enumerate(sym_net(theta, widths, lam)):
        ref = jets_of(e, PTS)
        assert np.allclose(got[:, k], ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("equation", [p2.IPM2D, p2.BOUSS2D])
def test_fields_match_sympy(tiny, equation):
    widths, theta = tiny
    lam = 1.3992
    if equation == p2.IPM2D:
        widths = widths[:-1] + [1]
        theta = theta[:sum(b * (a + 1) for a, b in zip(widths[:-1], widths[1:]))]
    y1 = np.array([p[0] for p in PTS])
    y2 = np.array([p[1] for p in PTS])
    got = p2.fields(theta, widths, y1, y2, lam, equation)
    for f, e in enumerate(sym_fields(theta, widths, lam, equation)):
        assert np.allclose(got[f], jets_of(e, PTS), rtol=1e-11, atol=1e-13)


def test_ipm_residual_and_derivative_rows_match_sympy(tiny):
    widths, theta = tiny
    widths = widths[:-1] + [1]
    theta = theta[:sum(b * (a + 1) for a, b in zip(widths[:-1], widths[1:]))]
    lam = 0.4721
    Phi = sym_fields(theta, widths, lam, p2.IPM2D)[0]
    R = Phi + ((1 + lam) * Y1 + Phi) * sp.diff(Phi, Y1) + (1 + lam) * Y2 * sp.diff(Phi, Y2)
    y1 = np.array([p[0] for p in PTS])
    y2 = np.array([p[1] for p in PTS])
    F = p2.fields(theta, widths, y1, y2, lam, p2.IPM2D)[0]
    assert np.allclose(p2.ipm_residual(F, y1, y2, lam), evaluate(R, PTS), rtol=1e-11, atol=1e-13)
    d1, d2 = p2.ipm_residual_d1(F, y1, y2, lam)
    assert np.allclose(d1, evaluate(sp.diff(R, Y1), PTS), rtol=1e-10, atol=1e-12)
    assert np.allclose(d2, evaluate(sp.diff(R, Y2), PTS), rtol=1e-10, atol=1e-12)
    # boundary rows: dPhi/dy2 on y2 = 0
    e1 = np.array([0.4, 2.0])
    Fe = p2.fields(theta, widths, e1, np.zeros(2), lam, p2.IPM2D)[0]
    assert np.allclose(Fe[2], evaluate(sp.diff(Phi, Y2), [(0.4, 0.0), (2.0, 0.0)]), rtol=1e-11, atol=1e-13)


def test_boussinesq_residuals_match_sympy(tiny):
    widths, theta = tiny
    lam = 1.3992
    Om, Th, Ps = sym_fields(theta, widths, lam, p2.BOUSS2D)
    U1, U2 = -sp.diff(Ps, Y2), sp.diff(Ps, Y1)
    V1, V2 = (1 + lam) * Y1 + U1, (1 + lam) * Y2 + U2
    Ro = Om + V1 * sp.diff(Om, Y1) + V2 * sp.diff(Om, Y2) - sp.diff(Th, Y1)
    Rt = (1 - lam) * Th + V1 * sp.diff(Th, Y1) + V2 * sp.diff(Th, Y2)
    Rp = sp.diff(Ps, Y1, 2) + sp.diff(Ps, Y2, 2) - Om
    y1 = np.array([p[0] for p in PTS])
    y2 = np.array([p[1] for p in PTS])
    F = p2.fields(theta, widths, y1, y2, lam, p2.BOUSS2D)
    got = p2.bouss_residuals(F[0], F[1], F[2], y1, y2, lam)
    for g, e in zip(got, (Ro, Rt, Rp)):
        assert np.allclose(g, evaluate(e, PTS), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("name", ["ipm2d", "bouss2d"])
def test_rows_layout_and_scaling(name):
    inp = workloads.make_inputs_2d(name, n=16, n1=4 if name == "ipm2d" else 0, ne=4,
                                   widths=[2, 4, 4, 1 if name == "ipm2d" else 3], nval=16)
    pr = p2.Problem.from_inputs(inp)
    th = inp["theta0"]
    r = pr.residual_rows(th)
    assert r.shape == (pr.m,)
    # equation rows of point 3
    R = pr.raw(th, pr.y1[3:4], pr.y2[3:4])
    for e in range(pr.n_eq):
        assert r[3 * pr.n_eq + e] == pytest.approx(np.sqrt(1.0 / (pr.n * pr.n_eq)) * R[e][0], rel=1e-14)
    # normalisation row
    nn0 = p2.mlp_jets(th, pr.widths, np.zeros(1), np.zeros(1), pr.lam)[0, 0, 0]
    assert r[-1] == pytest.approx(np.sqrt(pr.c_norm) * (nn0 - pr.c_target), rel=1e-14)
    # any subset of rows agrees with the full evaluation
    rows = np.array([0, pr.m // 2, pr.m - 2, pr.m - 1])
    assert np.allclose(pr.residual_rows(th, rows), r[rows], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("name", ["ipm2d", "bouss2d"])
def test_complex_step_jacobian(name):
    inp = workloads.make_inputs_2d(name, n=24, n1=6 if name == "ipm2d" else 0, ne=4,
                                   widths=[2, 5, 5, 1 if name == "ipm2d" else 3], nval=16)
    pr = p2.Problem.from_inputs(inp)
    th = inp["theta0"] + 0.1 * np.random.default_rng(1).standard_normal(pr.P)
    J = pr.jacobian(th)
    # central differences along random directions (truncation O(h^2))
    for seed in range(3):
        v = np.random.default_rng(10 + seed).standard_normal(pr.P)
        h = 1e-5
        fd = (pr.residual_rows(th + h * v) - pr.residual_rows(th - h * v)) / (2 * h)
        assert np.linalg.norm(J @ v - fd) <= 1e-8 * np.linalg.norm(fd)
    # the output bias enters NN_0 additively: its column is d r / d NN_0 applied to a constant
    k_bias0 = pr.P - pr.widths[-1]
    base = pr.residual_rows(th)
    t2 = th.copy()
    t2[k_bias0] += 1.0
    lin = pr.residual_rows(t2) - base  # exact up to the products with other NN_0 terms
    if name == "ipm2d":
        # R is quadratic in NN_0 (the Phi Phi_1 term); the second difference isolates it
        t3 = th.copy()
        t3[k_bias0] -= 1.0
        col = 0.5 * (pr.residual_rows(t2) - pr.residual_rows(t3))
        assert np.allclose(J[:, k_bias0], col, rtol=1e-9, atol=1e-12)
    else:
        assert np.allclose(J[:, k_bias0], lin, rtol=1e-9, atol=1e-12)  # linear in NN_0


def test_oracle_step_on_2d_problem():
    inp = workloads.make_inputs_2d("ipm2d", n=32, n1=8, ne=4, widths=[2, 6, 6, 1], nval=16)
    pr = p2.Problem.from_inputs(inp)
    th = inp["theta0"]
    nxt, st = ogn.step(pr, th, 1e-3)
    assert st["chol_info"] == 0
    assert ogn.backward_error(st["G"], 1e-3, st["g"], nxt - th) < 1e-14
    # the step minimises the damped model |r + J d|^2 + mu |d|^2, so it is below d = 0
    d, r, J = nxt - th, st["r"], st["J"]
    assert np.sum((r + J @ d) ** 2) + 1e-3 * d @ d < r @ r


def sym_residuals(theta, widths, lam, equation):
    """The residual expressions of each equation (sympy), from the fields."""
    F = sym_fields(theta, widths, lam, equation)
    if equation == p2.IPM2D:
        Phi = F[0]
        return [Phi + ((1 + lam) * Y1 + Phi) * sp.diff(Phi, Y1) + (1 + lam) * Y2 * sp.diff(Phi, Y2)]
    Om, Th, Ps = F
    V1, V2 = (1 + lam) * Y1 - sp.diff(Ps, Y2), (1 + lam) * Y2 + sp.diff(Ps, Y1)
    return [Om + V1 * sp.diff(Om, Y1) + V2 * sp.diff(Om, Y2) - sp.diff(Th, Y1),
            (1 - lam) * Th + V1 * sp.diff(Th, Y1) + V2 * sp.diff(Th, Y2),
            sp.diff(Ps, Y1, 2) + sp.diff(Ps, Y2, 2) - Om]


@pytest.mark.parametrize("equation", [p2.IPM2D, p2.BOUSS2D])
def test_validation_and_train_max_against_sympy(tiny, equation):
    """Paper: Methods, "Validation Metrics for Solutions" (max |R| over a
    grid).  Each grid point is mapped to y = s/(1-s) here and every
    equation's residual is evaluated symbolically; the maxima must agree, and
    the validation and collocation maxima must differ (an oracle that mixed up
    the two grids, or dropped an equation, fails)."""
    widths, theta = tiny
    name = "ipm2d" if equation == p2.IPM2D else "bouss2d"
    if equation == p2.IPM2D:
        widths = widths[:-1] + [1]
        theta = theta[:sum(b * (a + 1) for a, b in zip(widths[:-1], widths[1:]))]
    lam = workloads.WORKLOADS_2D[name]["lam"]
    inp = workloads.make_inputs_2d(name, n=8, n1=0, ne=2, widths=widths, nval=4)
    pr = p2.Problem.from_inputs(inp)
    exprs = sym_residuals(theta, widths, lam, equation)

    def brute(s):
        pts = [(a / (1 - a), b / (1 - b)) for a, b in s]
        return max(float(np.max(np.abs(evaluate(e, pts)))) for e in exprs)

    ref_val, ref_train = brute(inp["sval"]), brute(inp["s"])
    assert abs(pr.validation_max(theta) - ref_val) <= 1e-11 * ref_val
    assert abs(pr.train_max(theta) - ref_train) <= 1e-11 * ref_train
    assert abs(ref_val - ref_train) > 1e-6 * ref_val
    if equation == p2.BOUSS2D:
        # each equation's maximum differs, so dropping one would change the result
        pts = [(a / (1 - a), b / (1 - b)) for a, b in inp["sval"]]
        per = [float(np.max(np.abs(evaluate(e, pts)))) for e in exprs]
        assert len({round(v, 12) for v in per}) == 3
