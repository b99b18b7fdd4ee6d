"""Pins of the oracle's model half (oracle/profile1d.py) against mathematics
that does not go through the oracle's own formulas: complex-step derivatives,
closed-form Hilbert pairs, closed-form self-similar profiles, the
time-dependent equation the residual is reduced from, and the paper's printed
constants.  CPU only."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1

LAM = workloads.LAM_CCF1
H_CS = 1e-30  # complex-step increment


def cs(fun, x):
    """Complex-step derivative Im f(x + ih)/h (exact to rounding for analytic f)."""
    return np.imag(fun(np.asarray(x, dtype=np.complex128) + 1j * H_CS)) / H_CS


# ---------------------------------------------------------------------------
# Geometry and envelope
# ---------------------------------------------------------------------------
def test_map_inverts_compactified_coordinate():
    s = np.concatenate([[0.0, 1e-12, 1e-6], np.linspace(0.01, 0.999, 50), [1 - 1e-8]])
    q, y = p1.coords(s, LAM)
    # q = (1+y^2)^{-1/(2(1+lam))} is the paper's coordinate; coords must invert it
    np.testing.assert_allclose(p1.q_of_y(y, LAM), q, rtol=4e-15, atol=0)
    assert y[0] == 0.0 and np.all(np.diff(y) > 0)


def test_map_derivatives_by_complex_step():
    s = np.linspace(0.02, 0.98, 40)
    np.testing.assert_allclose(p1.dy_ds(s, LAM), cs(lambda z: p1.coords(z, LAM)[1], s), rtol=1e-13)
    y = np.geomspace(1e-3, 1e6, 40)
    np.testing.assert_allclose(p1.dq_dy(y, LAM), cs(lambda z: p1.q_of_y(z, LAM), y), rtol=1e-13)


@pytest.mark.parametrize("eq", [p1.CCF, p1.BURGERS])
def test_envelope_derivative_and_shape(eq):
    y = np.geomspace(1e-4, 1e8, 60)
    E, Ey = p1.envelope(y, LAM, eq)
    np.testing.assert_allclose(Ey, cs(lambda z: p1.envelope(z, LAM, eq)[0], y), rtol=1e-13)
    qneg = p1.q_of_y(y, LAM) ** (-LAM)
    if eq == p1.CCF:
        # even, ~ y^2 at the origin, ~ q^{-lam} in the far field
        np.testing.assert_allclose(p1.envelope(-y, LAM, eq)[0], E, rtol=0)
        assert abs(E[0] / y[0] ** 2 - 1) < 1e-7
    else:
        np.testing.assert_allclose(p1.envelope(-y, LAM, eq)[0], -E, rtol=0)
        assert abs(E[0] / y[0] - 1) < 1e-7
    assert abs(E[-1] / qneg[-1] - 1) < 1e-12


# ---------------------------------------------------------------------------
# Network jets
# ---------------------------------------------------------------------------
def test_one_neuron_closed_form():
    w1, b1, w2, b2 = 0.7, -0.2, 1.3, 0.4
    theta = np.array([w1, b1, w2, b2])
    x = np.linspace(0, 1, 11)
    NN, NNx, _ = p1.mlp_jets(theta, [1, 1, 1], x)
    np.testing.assert_allclose(NN, w2 * np.tanh(w1 * x + b1) + b2, rtol=1e-15)
    np.testing.assert_allclose(NNx, w2 * w1 / np.cosh(w1 * x + b1) ** 2, rtol=1e-14)


def test_input_jet_by_complex_step():
    widths = [1, 16, 16, 1]
    theta = workloads.glorot_theta(widths, 7)
    x = np.linspace(0.0, 1.0, 33)
    _, NNx, _ = p1.mlp_jets(theta, widths, x)
    np.testing.assert_allclose(NNx, cs(lambda z: p1.mlp_jets(theta, widths, z)[0], x), rtol=1e-13, atol=1e-15)


def test_param_rows_by_complex_step():
    widths = [1, 8, 8, 1]
    theta = workloads.glorot_theta(widths, 3)
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, 9)
    s0, s1 = rng.standard_normal(9), rng.standard_normal(9)
    rows = p1.mlp_param_rows(theta, widths, x, s0, s1)
    ref = np.zeros_like(rows)
    for p in range(theta.size):
        e = np.zeros(theta.size, dtype=np.complex128)
        e[p] = 1j * H_CS
        NN, NNx, _ = p1.mlp_jets(theta + e, widths, x.astype(np.complex128))
        ref[:, p] = (s0 * NN.imag + s1 * NNx.imag) / H_CS
    np.testing.assert_allclose(rows, ref, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Hilbert transform on the half line (even functions)
# ---------------------------------------------------------------------------
def _hilbert_setup(m=1024, lam=LAM):
    sq, wq = workloads.quadrature_s(m)
    t, what = p1.hilbert_weights(sq, wq, lam)
    x = p1.coords(np.linspace(0.001, 0.95, 200), lam)[1]
    return t, what, x, p1.hilbert_matrix(x, t, what)


@pytest.mark.parametrize("fun,ref,tol", [
    (lambda s: 1 / (1 + s * s), lambda x: x / (1 + x * x), 1e-10),
    (lambda s: s * s / (1 + s * s), lambda x: -x / (1 + x * x), 1e-10),
    # integrand ~ q^{0.12} at s -> 1 (an endpoint singularity): slower convergence
    (lambda s: np.abs(s) ** 0.3, lambda x: -np.tan(np.pi * 0.3 / 2) * np.abs(x) ** 0.3, 1e-5),
])
def test_hilbert_closed_forms(fun, ref, tol):
    # H f(x) = (1/pi) p.v. int f(s)/(x - s) ds; the listed pairs are classical
    t, what, x, Q = _hilbert_setup()
    U = p1.hilbert_even(Q, fun(t), fun(x))
    scale = np.maximum(1.0, np.abs(ref(x)))
    assert np.max(np.abs(U - ref(x)) / scale) < tol


# ---------------------------------------------------------------------------
# Residual operator
# ---------------------------------------------------------------------------
def test_selfsimilar_reduction_of_ccf():
    """theta(x,t) = (1-t)^lam Theta(x (1-t)^{-(1+lam)}) in theta_t + (H theta) theta_x
    equals (1-t)^{lam-1} R[Theta](y).  Theta = y^2/(1+y^2), H Theta = -y/(1+y^2)
    (classical pair); theta_t by complex step in t, theta_x by complex step in x."""
    lam = 0.6057
    Th = lambda y: y * y / (1 + y * y)
    HTh = lambda y: -y / (1 + y * y)
    x, t = np.linspace(-3, 3, 31), 0.37
    phys = lambda xx, tt: (1 - tt) ** lam * Th(xx * (1 - tt) ** (-(1 + lam)))
    th_t = cs(lambda tt: phys(x, tt), np.full_like(x, t))
    th_x = cs(lambda xx: phys(xx, t), x)
    y = x * (1 - t) ** (-(1 + lam))
    H_phys = (1 - t) ** lam * HTh(y)  # H commutes with dilations
    lhs = th_t + H_phys * th_x
    Thy = cs(Th, y)
    rhs = (1 - t) ** (lam - 1) * p1.residual_operator(lam, y, Th(y), Thy, HTh(y))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-14)


def test_burgers_closed_form_profile_has_zero_residual():
    """lam = 1/2: U^3 + U + y = 0 solves -lam U + ((1+lam) y + U) U' = 0 (the
    Burgers illustration of the paper's research-flowchart figure)."""
    lam = 0.5
    y = np.linspace(-5, 5, 101)
    U = np.array([np.real(r[np.abs(r.imag) < 1e-9][0]) for r in (np.roots([1, 0, 1, yy]) for yy in y)])
    Uy = -1.0 / (3 * U * U + 1)
    R = p1.residual_operator(lam, y, U, Uy, U)
    assert np.max(np.abs(R)) < 1e-14


def test_paper_printed_constants():
    """alpha threshold 1/(1+lambda) printed in the CCF paragraph pins the
    exponent convention y = x (1-t)^{-(1+lambda)} used by the coordinate map."""
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    assert round(1 / (1 + d["ccf_lambda_1"]), 3) == d["ccf_alpha_1_printed"]
    assert round(1 / (1 + d["ccf_lambda_2"]), 2) == d["ccf_alpha_2_printed"]
    # far-field growth of the CCF envelope is the homogeneous solution of
    # -lam Theta + (1+lam) y Theta' = 0, i.e. |y|^{lam/(1+lam)}
    y = np.array([1e6, 1e9])
    E, Ey = p1.envelope(y, d["ccf_lambda_1"], p1.CCF)
    lam = d["ccf_lambda_1"]
    assert np.max(np.abs(-lam * E + (1 + lam) * y * Ey) / E) < 1e-9


# ---------------------------------------------------------------------------
# Jacobian of the residual rows
# ---------------------------------------------------------------------------
def _small_problem(eq, n=96, m=96, widths=(1, 8, 8, 1), seed=5):
    inp = workloads.make_inputs("ccf_small", n=n, m_quad=m, widths=widths)
    inp["theta0"] = workloads.glorot_theta(widths, seed)
    return p1.Problem.from_inputs(inp, equation=eq), inp["theta0"]


@pytest.mark.parametrize("eq", [p1.CCF, p1.BURGERS])
def test_jacobian_by_complex_step(eq):
    prob, theta = _small_problem(eq)
    J = p1.jacobian(prob, theta)
    ref = np.zeros_like(J)
    for p in range(theta.size):
        e = np.zeros(theta.size, dtype=np.complex128)
        e[p] = 1j * H_CS
        ref[:, p] = p1.residual_rows(prob, theta + e).imag / H_CS
    assert np.linalg.norm(J - ref) / np.linalg.norm(ref) < 1e-13


def test_jacobian_rows_subset_and_central_differences():
    prob, theta = _small_problem(p1.CCF, widths=(1, 12, 12, 1))
    J = p1.jacobian(prob, theta)
    rows = np.array([0, 5, 50, prob.n])
    np.testing.assert_allclose(p1.jacobian(prob, theta, rows=rows), J[rows], rtol=1e-13, atol=1e-16)
    h = 1e-6
    v = workloads.perturbation(theta.size, 11)
    fd = (p1.residual_rows(prob, theta + h * v) - p1.residual_rows(prob, theta - h * v)) / (2 * h)
    assert np.linalg.norm(J @ v - fd) / np.linalg.norm(fd) < 1e-7


def test_row_zero_at_origin_is_zero_for_ccf():
    prob, theta = _small_problem(p1.CCF)
    assert prob.s[0] == 0.0
    J = p1.jacobian(prob, theta, rows=[0])
    assert np.all(J == 0.0)


@pytest.mark.parametrize("eq", [p1.CCF, p1.BURGERS])
def test_teacher_zero_is_reached_to_second_order(eq):
    """With the source f = R[NN_theta*] and c_target = NN_theta*(1), theta* is an
    exact zero of r.  One damped GN step from theta* + eps v leaves a residual
    of order eps^2 (it is order eps if J is wrong in any term): going from
    eps = 1e-2 to 1e-3 must shrink it by far more than 10x."""
    prob, tstar = _small_problem(eq, n=160, m=128, widths=(1, 8, 8, 1), seed=9)
    R, _ = p1.raw_residual(prob, tstar)
    prob.f = R.copy()
    NN1, _, _ = p1.mlp_jets(tstar, prob.widths, np.ones(1))
    prob.c_target = NN1[0]
    assert np.linalg.norm(p1.residual_rows(prob, tstar)) == 0.0
    v = workloads.perturbation(tstar.size, 2)
    after = []
    for eps in (1e-2, 1e-3):
        th1, st = ogn.step(prob, tstar + eps * v, 1e-8)
        assert st["chol_info"] == 0
        after.append(np.linalg.norm(p1.residual_rows(prob, th1)))
    assert after[0] / after[1] > 40
    assert after[1] < 1e-6
