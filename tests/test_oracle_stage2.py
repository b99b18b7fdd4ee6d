"""Pins of the second-stage oracle (oracle/stage2.py): the exact quadratic
expansion R[Theta_1 + eps Theta_2] = R[Theta_1] + eps D[Theta_1] Theta_2 +
eps^2 U[Theta_2] Theta_2' checked against residuals of the summed field
computed independently (CCF and the local variant); the Fourier feature
jets against a complex-step derivative in the input; the complex-step
Jacobian against central differences; a manufactured stage-2 zero reached
by Gauss-Newton to rounding.  CPU only."""
import numpy as np
import pytest

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1
from oracle import stage2 as s2

LAM = 0.6057


def _setup(equation, n=90, widths2=(8, 6, 1), F=4, eps=1e-3, seed=7):
    inp = workloads.make_inputs("ccf_small", n=n, m_quad=48, widths=[1, 6, 6, 1])
    if equation == p1.BURGERS:
        inp["c_target"] = -1.0
    base = p1.Problem.from_inputs(inp, equation=equation)
    rng = np.random.default_rng(seed)
    b = rng.normal(0.0, 2 * np.pi * 3.0, size=F)
    widths2 = [2 * F] + list(widths2[1:])
    theta2 = workloads.glorot_theta(widths2, seed + 1)
    prob = s2.Stage2Problem(base, inp["theta0"], widths2, b, eps)
    return inp, base, prob, theta2


def _summed_residual(base, theta1, prob, theta2, eps):
    """R of Theta_1 + eps Theta_2 from the two fields, independently of prob.linearised."""
    T1, T1y, _ = p1.field(theta1, base.widths, base.y, base.lam, base.equation)
    T2, T2y = prob.field2(theta2, base.y)
    Th, Thy = T1 + eps * T2, T1y + eps * T2y
    if base.equation == p1.CCF:
        t1, _, _ = p1.field(theta1, base.widths, base.t, base.lam, base.equation)
        t2, _ = prob.field2(theta2, base.t)
        U = p1.hilbert_even(base.Q, t1 + eps * t2, Th)
        U2 = p1.hilbert_even(base.Q, t2, T2)
    else:
        U, U2 = Th, T2
    return p1.residual_operator(base.lam, base.y, Th, Thy, U), U2 * T2y


@pytest.mark.parametrize("equation", [p1.CCF, p1.BURGERS])
def test_exact_quadratic_expansion(equation):
    inp, base, prob, theta2 = _setup(equation)
    D = prob.linearised(theta2)
    for eps in (1e-1, 1e-3):
        R, quad = _summed_residual(base, inp["theta0"], prob, theta2, eps)
        lhs = R - prob.R1
        rhs = eps * D + eps * eps * quad
        assert np.max(np.abs(lhs - rhs)) < 1e-12 * max(1.0, np.max(np.abs(R)))


def test_fourier_jets_by_complex_step():
    F = 5
    b = np.random.default_rng(3).normal(0, 8.0, F)
    widths = [2 * F, 7, 4, 1]
    theta = workloads.glorot_theta(widths, 5)
    x = np.linspace(0.05, 1.0, 11)
    NN, NNx = s2.fourier_mlp_jets(theta, widths, b, x)
    h = 1e-30
    NNc, _ = s2.fourier_mlp_jets(theta, widths, b, x + 1j * h)
    np.testing.assert_allclose(NNx, np.imag(NNc) / h, rtol=1e-13, atol=1e-14)
    phi, dphi = s2.fourier_features(np.array([0.3]), b)
    np.testing.assert_allclose(phi[:F, 0], np.cos(0.3 * b), rtol=1e-15)
    np.testing.assert_allclose(dphi[F:, 0], b * np.cos(0.3 * b), rtol=1e-15)


@pytest.mark.parametrize("equation", [p1.CCF, p1.BURGERS])
def test_jacobian_against_central_differences(equation):
    inp, base, prob, theta2 = _setup(equation, widths2=(6, 5, 1), F=3)
    J = prob.jacobian(theta2)
    rng = np.random.default_rng(9)
    for _ in range(3):
        v = rng.standard_normal(theta2.size)
        h = 1e-6
        fd = (prob.residual_rows(theta2 + h * v) - prob.residual_rows(theta2 - h * v)) / (2 * h)
        np.testing.assert_allclose(J @ v, fd, rtol=1e-6, atol=1e-10)


def test_manufactured_stage2_zero_is_reached():
    """With R_1 := -eps D[Theta_1] Theta_2(theta2*), theta2* zeroes every row.  One
    GN step from theta2* + e v leaves a residual of order e^2 (order e if J were
    wrong in any term): from e = 1e-2 to 1e-3 it must shrink by far more than 10x."""
    inp, base, prob, theta2 = _setup(p1.CCF, widths2=(6, 5, 1), F=3, eps=1e-2)
    prob.R1 = -prob.eps * prob.linearised(theta2)
    base.c_norm = 0.0
    assert np.max(np.abs(prob.residual_rows(theta2))) < 1e-15
    v = workloads.perturbation(theta2.size, 4)
    after = []
    for e in (1e-2, 1e-3):
        th, st = ogn.step(prob, theta2 + e * v, 1e-14)
        after.append(np.linalg.norm(prob.residual_rows(th)))
    assert after[0] / after[1] > 40
    th = theta2 + 1e-2 * v
    for _ in range(6):
        th, st = ogn.step(prob, th, 1e-14)
    assert np.linalg.norm(prob.residual_rows(th)) < 1e-9
