"""Pins of the d1/d2-row oracle (oracle/deriv1d.py): Taylor-mode field
derivatives against sympy's symbolic derivatives of the same composite
Theta(y); the odd-function Hilbert quadrature against classical pairs; the
R' and R'' formulas against symbolic derivatives of the residual for the
manufactured CCF pair Theta = y^2/(1+y^2), H Theta = -y/(1+y^2) and for the
local Burgers form; the whole d1 row of the local variant against a
complex-step derivative in y of its d0 residual; the complex-step Jacobian
against central differences; the row layout.  CPU only."""
import numpy as np
import pytest
import sympy as sp

import workloads
from oracle import deriv1d as d1
from oracle import gn as ogn
from oracle import profile1d as p1

LAM = 0.6057


def _sym_field(theta, widths, lam, equation):
    ys = sp.Symbol("y", positive=True)
    w = 1 + ys ** 2
    h = [w ** (-1 / (2 * (1 + sp.Float(lam, 30))))]     # q(y)
    layers = p1.unpack(theta, widths)
    for l, (W, b) in enumerate(layers):
        z = [sum(sp.Float(W[i, j], 30) * h[j] for j in range(W.shape[1])) + sp.Float(b[i], 30)
             for i in range(W.shape[0])]
        h = [sp.tanh(v) for v in z] if l < len(layers) - 1 else z
    e = sp.Float(lam, 30) / (2 * (1 + sp.Float(lam, 30)))
    E = ys ** 2 * w ** (e - 1) if equation == p1.CCF else ys * w ** (e - sp.Rational(1, 2))
    return ys, E * h[0]


@pytest.mark.parametrize("equation", [p1.CCF, p1.BURGERS])
def test_field_derivatives_match_sympy(equation):
    widths = [1, 3, 2, 1]
    theta = workloads.glorot_theta(widths, 4) + 0.1
    ys, Th = _sym_field(theta, widths, LAM, equation)
    yv = np.array([0.05, 0.7, 2.3, 11.0])
    F = d1.field_derivs(theta, widths, yv, LAM, equation)
    for k in range(4):
        expr = sp.diff(Th, ys, k)
        ref = np.array([float(expr.subs(ys, v).evalf(30)) for v in yv])
        np.testing.assert_allclose(F[k], ref, rtol=1e-11, atol=1e-14)


def test_taylor_power_is_the_binomial_series():
    a = d1.tvar(np.array([0.0]))
    a[0] += 1.0                     # 1 + y at y = 0
    u = d1.tpow(a, 0.37)
    ref = [1.0, 0.37, 0.37 * (0.37 - 1) / 2, 0.37 * (0.37 - 1) * (0.37 - 2) / 6]
    np.testing.assert_allclose(u[:, 0], ref, rtol=1e-15)


@pytest.mark.parametrize("fun,ref,tol", [
    # d/dx of the classical even pair H[1/(1+s^2)] = x/(1+x^2)
    (lambda s: -2 * s / (1 + s * s) ** 2, lambda x: (1 - x * x) / (1 + x * x) ** 2, 1e-9),
    # H[s/(1+s^2)] = -1/(1+x^2) (H H = -I applied to the even pair)
    (lambda s: s / (1 + s * s), lambda x: -1 / (1 + x * x), 1e-9),
])
def test_odd_hilbert_closed_forms(fun, ref, tol):
    sq, wq = workloads.quadrature_s(1024)
    t, what = p1.hilbert_weights(sq, wq, LAM)
    x = p1.coords(np.linspace(0.001, 0.95, 200), LAM)[1]
    U = d1.hilbert_odd(x, t, what, fun(t), fun(x))
    assert np.max(np.abs(U - ref(x)) / np.maximum(1.0, np.abs(ref(x)))) < tol


def test_residual_derivative_formulas_ccf_manufactured():
    ys = sp.Symbol("y", positive=True)
    lam = sp.Float(LAM, 30)
    Th, U = ys ** 2 / (1 + ys ** 2), -ys / (1 + ys ** 2)
    R = -lam * Th + ((1 + lam) * ys + U) * sp.diff(Th, ys)
    yv = np.array([0.1, 0.8, 1.7, 6.0])
    ev = lambda e: np.array([float(e.subs(ys, v)) for v in yv])
    F = np.stack([ev(sp.diff(Th, ys, k)) for k in range(4)])
    R1, R2 = d1.residual_derivs(LAM, yv, F, ev(U), ev(sp.diff(U, ys)), ev(sp.diff(U, ys, 2)))
    np.testing.assert_allclose(R1, ev(sp.diff(R, ys)), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(R2, ev(sp.diff(R, ys, 2)), rtol=1e-13, atol=1e-15)


def test_residual_derivative_formulas_burgers():
    ys = sp.Symbol("y", positive=True)
    lam = sp.Rational(1, 2)
    U = ys / sp.sqrt(1 + ys ** 2) * (1 + ys ** 2) ** sp.Rational(1, 6)
    R = -lam * U + ((1 + lam) * ys + U) * sp.diff(U, ys)
    yv = np.array([0.2, 1.1, 3.0])
    ev = lambda e: np.array([float(e.subs(ys, v)) for v in yv])
    F = np.stack([ev(sp.diff(U, ys, k)) for k in range(4)])
    R1, R2 = d1.residual_derivs(0.5, yv, F, F[0], F[1], F[2])
    np.testing.assert_allclose(R1, ev(sp.diff(R, ys)), rtol=1e-13)
    np.testing.assert_allclose(R2, ev(sp.diff(R, ys, 2)), rtol=1e-13)


def _small(equation, n=60, n1=17, n2=13, widths=(1, 6, 5, 1)):
    inp = workloads.make_inputs("ccf_small", n=n, m_quad=48, widths=list(widths))
    if equation == p1.BURGERS:
        inp["c_target"] = -1.0
    base = p1.Problem.from_inputs(inp, equation=equation)
    s1 = (np.arange(n1) + 0.5) / n1 * 0.97
    s2 = (np.arange(n2) + 0.25) / n2 * 0.97
    return inp, d1.Problem(base, s1, s2, c_d1=0.7, c_d2=0.3)


def test_burgers_d1_row_is_the_y_derivative_of_the_residual():
    inp, prob = _small(p1.BURGERS)
    theta = inp["theta0"]
    _, y1 = p1.coords(prob.s1, prob.lam)
    h = 1e-30
    Rc, _ = p1.raw_residual(prob, theta.astype(np.complex128), y=y1 + 1j * h)
    R1, _ = d1.deriv_residuals(prob, theta, prob.s1, None)
    np.testing.assert_allclose(R1, np.imag(Rc) / h, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("equation", [p1.CCF, p1.BURGERS])
def test_rows_layout(equation):
    inp, prob = _small(equation)
    theta = inp["theta0"]
    r = prob.residual_rows(theta)
    assert r.size == prob.n + prob.n1 + prob.n2 + 1 == prob.m
    base = p1.residual_rows(prob, theta)
    np.testing.assert_array_equal(r[:prob.n], base[:prob.n])
    assert r[-1] == base[-1]
    R1, R2 = d1.deriv_residuals(prob, theta, prob.s1, prob.s2)
    np.testing.assert_allclose(r[prob.n:prob.n + prob.n1], np.sqrt(0.7 / prob.n1) * R1, rtol=1e-15)
    np.testing.assert_allclose(r[prob.n + prob.n1:-1], np.sqrt(0.3 / prob.n2) * R2, rtol=1e-15)


@pytest.mark.parametrize("equation", [p1.CCF, p1.BURGERS])
def test_complex_step_jacobian_against_central_differences(equation):
    inp, prob = _small(equation, widths=(1, 4, 3, 1))
    theta = inp["theta0"]
    J = prob.jacobian(theta)
    rng = np.random.default_rng(12)
    for _ in range(4):
        v = rng.standard_normal(theta.size)
        h = 1e-6
        fd = (prob.residual_rows(theta + h * v) - prob.residual_rows(theta - h * v)) / (2 * h)
        np.testing.assert_allclose(J @ v, fd, rtol=1e-6, atol=1e-8)
    # the d0 and normalisation rows agree with the analytic Jacobian of the d0 problem
    J0 = p1.jacobian(prob, theta, rows=np.arange(prob.n + 1))   # d0 rows, then the normalisation row
    np.testing.assert_allclose(J[:prob.n], J0[:prob.n], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(J[-1], J0[prob.n], rtol=1e-14, atol=1e-15)


def test_step_with_derivative_rows_decreases_the_model():
    inp, prob = _small(p1.CCF, widths=(1, 5, 5, 1))
    th, st = ogn.step(prob, inp["theta0"], 1e-3)
    r, J, d = st["r"], st["J"], st["delta"]
    assert float(np.sum((r + J @ d) ** 2)) < float(r @ r)


def test_lambda_estimate_reads_the_odd_transform_at_the_origin():
    # Theta = y^2/(1+y^2): H[Theta'] = d/dy (-y/(1+y^2)), which is -1 at 0, so lam_hat = 0;
    # the same through the odd quadrature directly, and an affine check on the formula
    sq, wq = workloads.quadrature_s(1024)
    t, what = p1.hilbert_weights(sq, wq, LAM)
    dth = lambda s: 2 * s / (1 + s * s) ** 2
    U1_0 = d1.hilbert_odd(np.zeros(1), t, what, dth(t), np.zeros(1))[0]
    assert U1_0 == pytest.approx(-1.0, abs=1e-9)
    inp, prob = _small(p1.CCF)
    lam_hat, u = d1.lambda_estimate(prob, inp["theta0"])
    assert lam_hat == pytest.approx(-2.0 * (1.0 + u), rel=1e-15)
    # U'(0) equals the limit of U'(y) from the d1 machinery at small y
    F = d1.field_derivs(inp["theta0"], prob.widths, np.array([1e-7]), prob.lam, prob.equation)
    _, U1, _ = d1.transform_derivs(prob, inp["theta0"], np.array([1e-7]), F)
    assert U1[0] == pytest.approx(u, rel=1e-6, abs=1e-9)
