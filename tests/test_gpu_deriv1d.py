"""GPU parity of the 1D derivative (d1, d2) rows against the oracle
(oracle/deriv1d.py: Taylor-mode field derivatives, odd and even half-line
Hilbert quadrature, complex-step Jacobian) on identical seeded inputs.
Tolerances as for the d0 rows: r, J, J^T v relative 1e-12 (normwise); the
step by backward error <= 5e-14 and forward error <= max(1e-12, 10 kappa
eps).  Cases: CCF with d1 and d2 rows (ragged counts, several tiles of the
jet sweep), the local variant with d1 rows only, a deeper CCF network with
d2 rows only, CCF with enough derivative rows for their coupling product to
run on a work plan (K split into pieces summed in a second launch); the
argument checks."""
import numpy as np
import pytest
import torch

import workloads
from oracle import deriv1d as d1
from oracle import gn as ogn
from oracle import profile1d as p1
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps

CASES = {
    "ccf_d1d2": (p1.CCF, dict(n=300, m_quad=64, widths=[1, 12, 10, 1]), 37, 29),
    "burgers_d1": (p1.BURGERS, dict(n=200, widths=[1, 8, 8, 1]), 50, 0),
    "ccf_deep_d2": (p1.CCF, dict(n=150, m_quad=40, widths=[1, 16, 16, 16, 1]), 0, 23),
    # 370 derivative rows x P = 673: 66 tiles of 64 x 64 in the derivative
    # rows' coupling product, which then runs on its work plan (every tile
    # split in 4 K pieces of its K = 3 m_quad = 192)
    "ccf_d1d2_planned": (p1.CCF, dict(n=300, m_quad=64, widths=[1, 24, 24, 1]), 200, 170),
}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def build(key):
    eq, over, n1, n2 = CASES[key]
    inp = workloads.make_inputs("ccf_small", **over)
    if eq == p1.BURGERS:
        inp["c_target"] = -1.0
    s1 = (np.arange(n1) + 0.5) / max(n1, 1) * 0.98
    s2 = (np.arange(n2) + 0.3) / max(n2, 1) * 0.98
    base = p1.Problem.from_inputs(inp, equation=eq)
    po = d1.Problem(base, s1, s2, c_d1=0.8, c_d2=0.4)
    pg = gn.Problem(eq, inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    ccf = eq == p1.CCF
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"] if ccf else None, inp["wq"] if ccf else None,
                  inp["sval"], s1=s1 if n1 else None, s2=s2 if n2 else None, c_d1=0.8, c_d2=0.4)
    return inp, po, pg


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[gpu deriv1d] case {request.param}", flush=True)
    inp, po, pg = build(request.param)
    theta = inp["theta0"] + 0.05 * np.random.default_rng(3).standard_normal(po.P)
    r = po.residual_rows(theta)
    J = po.jacobian(theta)
    yield dict(inp=inp, po=po, pg=pg, theta=theta, r=r, J=J)
    pg.close()


def test_rows_and_residual(case):
    po, pg = case["po"], case["pg"]
    assert pg.m == po.m
    r = pg.residual(dev(case["theta"])).cpu().numpy()
    assert rel(r, case["r"]) < 1e-12
    n = po.n
    # the derivative rows alone
    assert rel(r[n:-1], case["r"][n:-1]) < 1e-12


def test_jacobian(case):
    po, pg = case["po"], case["pg"]
    J, r = pg.jacobian(dev(case["theta"]))
    J = J.cpu().numpy()
    assert rel(J, case["J"]) < 1e-12
    n = po.n
    assert rel(J[n:-1], case["J"][n:-1]) < 1e-12
    assert rel(r.cpu().numpy(), case["r"]) < 1e-12


def test_vjp(case):
    po, pg = case["po"], case["pg"]
    v = np.random.default_rng(4).standard_normal(po.m)
    got = pg.vjp(dev(case["theta"]), dev(v)).cpu().numpy()
    assert rel(got, case["J"].T @ v) < 1e-12


def test_step(case):
    po, pg = case["po"], case["pg"]
    theta, mu = case["theta"], 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK
    ref, ost = ogn.step(po, theta, mu)
    d, dref = t.cpu().numpy() - theta, ref - theta
    G, g = ost["G"], ost["g"]
    assert ogn.backward_error(G, mu, g, d) < 5e-14
    kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
    assert rel(d, dref) < max(1e-12, 10 * kappa * EPS)
    assert st["half_sq_norm"] == pytest.approx(ost["half_sq_norm"], rel=1e-12)
    ev = pg.eval(dev(theta))
    assert ev["half_sq_norm"] == pytest.approx(ost["half_sq_norm"], rel=1e-12)


def test_argument_checks():
    inp = workloads.make_inputs("ccf_small", n=100, m_quad=32, widths=[1, 8, 1])
    pg = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    with pytest.raises(gn.GNError) as e:
        pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"], s1=np.array([0.5]),
                      c_d1=-1.0)
    assert e.value.status == gn.GN_EINVAL
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"], s1=np.array([0.2, 0.5]))
    assert pg.m == 100 + 2 + 1
    with pytest.raises(gn.GNError):
        gn.Batch([pg])
    pg.close()


def test_lambda_estimate(case):
    po, pg = case["po"], case["pg"]
    if po.equation != p1.CCF:
        with pytest.raises(gn.GNError):
            pg.lambda_estimate(dev(case["theta"]))
        return
    lam, du = pg.lambda_estimate(dev(case["theta"]))
    ref_lam, ref_du = d1.lambda_estimate(po, case["theta"])
    assert du == pytest.approx(ref_du, rel=1e-12, abs=1e-15)
    assert lam == pytest.approx(ref_lam, rel=1e-12, abs=1e-15)


def test_validation_derivative_maxima(case):
    po, pg, theta = case["po"], case["pg"], case["theta"]
    m1, m2 = pg.eval_derivs(dev(theta))
    R1, R2 = d1.deriv_residuals(po, theta, po.sval, po.sval)
    assert m1 == pytest.approx(np.max(np.abs(R1)), rel=1e-12)
    assert m2 == pytest.approx(np.max(np.abs(R2)), rel=1e-12)
