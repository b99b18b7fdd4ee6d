"""GPU parity of the 2D problems (IPM-style and Boussinesq-type stand-ins)
against the CPU oracle (oracle/profile2d.py: Taylor-mode jets, complex-step
Jacobian) on identical seeded inputs.  Tolerances as for the 1D path:
r, J, J^T v, max|R|: relative 1e-12 (normwise); the solve by backward error
<= 5e-14 and forward error <= max(1e-12, 10 kappa eps).  Cases span several
tiles of the jet sweep, ragged widths, three output fields and streamed row
chunks (the Gram accumulated over chunks, FP64 and split)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile2d as p2
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps

CASES = {
    "ipm_small": ("ipm2d", dict(n=64, n1=16, ne=8, widths=[2, 12, 12, 1], nval=64), {}),
    "ipm_ragged": ("ipm2d", dict(n=100, n1=30, ne=5, widths=[2, 20, 17, 9, 1], nval=36), {}),
    "bouss_small": ("bouss2d", dict(n=60, ne=8, widths=[2, 10, 10, 3], nval=64), {}),
    "bouss_chunked": ("bouss2d", dict(n=70, ne=6, widths=[2, 9, 11, 3], nval=16), dict(row_chunk=37)),
}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def build(key, precision="fp64"):
    name, over, extra = CASES[key]
    inp = workloads.make_inputs_2d(name, **over)
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                    precision=precision, row_chunk=extra.get("row_chunk", 0))
    pg.set_points_2d(inp["s"], inp["s1"] if inp["n1"] else None, inp["se"], inp["sval"])
    return inp, po, pg


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    print(f"\n[gpu 2d] case {request.param}", flush=True)
    inp, po, pg = build(request.param)
    theta = inp["theta0"] + 0.05 * np.random.default_rng(2).standard_normal(po.P)
    r = po.residual_rows(theta)
    J = po.jacobian(theta)
    G, g = ogn.gram_and_gradient(J, r)
    yield dict(key=request.param, inp=inp, po=po, pg=pg, theta=theta, r=r, J=J, G=G, g=g)
    pg.close()


def test_rows_count(case):
    assert case["pg"].m == case["po"].m


def test_residual(case):
    r = case["pg"].residual(dev(case["theta"])).cpu().numpy()
    assert rel(r, case["r"]) < 1e-12


def test_eval_stats(case):
    po, theta = case["po"], case["theta"]
    st = case["pg"].eval(dev(theta))
    assert abs(st["max_abs_R"] - po.train_max(theta)) <= 1e-12 * po.train_max(theta)
    assert abs(st["max_abs_R_val"] - po.validation_max(theta)) <= 1e-12 * po.validation_max(theta)
    h = 0.5 * case["r"] @ case["r"]
    assert abs(st["half_sq_norm"] - h) <= 1e-12 * h


def test_jacobian(case):
    J, r = case["pg"].jacobian(dev(case["theta"]), ld=case["po"].P + 3)
    assert rel(J.cpu().numpy(), case["J"]) < 1e-12
    assert rel(r.cpu().numpy(), case["r"]) < 1e-12


def test_step(case):
    po, pg, theta = case["po"], case["pg"], case["theta"]
    mu = 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1 and st["chol_info"] == 0
    d = t.cpu().numpy() - theta
    G, g = case["G"], case["g"]
    assert ogn.backward_error(G, mu, g, d) < 5e-14
    dref, info = ogn.damped_solve(G, g, mu)
    kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
    assert rel(d, dref) < max(1e-12, 10 * kappa * EPS)
    assert abs(st["half_sq_norm"] - 0.5 * case["r"] @ case["r"]) <= 1e-12 * (0.5 * case["r"] @ case["r"])


def test_vjp_and_autograd(case):
    pg, theta, J = case["pg"], case["theta"], case["J"]
    v = np.random.default_rng(3).standard_normal(J.shape[0])
    out = pg.vjp(dev(theta), dev(v)).cpu().numpy()
    assert rel(out, J.T @ v) < 1e-12
    th = dev(theta).requires_grad_(True)
    r = gn.residual(th, pg)
    (0.5 * (r * r).sum()).backward()
    assert rel(th.grad.cpu().numpy(), case["g"]) < 1e-12


def test_split_step_chunked():
    """Split-precision Gram accumulated over streamed row chunks."""
    inp, po, pg = build("bouss_chunked", precision="split32")
    theta = inp["theta0"]
    r = po.residual_rows(theta)
    J = po.jacobian(theta)
    G, g = ogn.gram_and_gradient(J, r)
    mu = 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK
    d = t.cpu().numpy() - theta
    dref, _ = ogn.damped_solve(G, g, mu)
    kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
    # the Gram carries ~1e-7 relative error from the FP32 products
    assert rel(d, dref) < 1e-6 * kappa
    pg.close()


def test_autograd_matches_central_differences():
    """Backward through the autograd Function against central differences
    (h = 1e-6) on 32 random unit parameter directions (IPM-style problem)."""
    inp, po, pg = build("ipm_small")
    theta = dev(inp["theta0"])
    th = theta.clone().requires_grad_(True)
    r = gn.residual(th, pg)
    L = 0.5 * (r * r).sum()
    L.backward()
    grad = th.grad.cpu().numpy()
    rng = np.random.default_rng(33)
    h = 1e-6
    for _ in range(32):
        d = rng.standard_normal(po.P)
        d /= np.linalg.norm(d)
        dd = dev(d)
        lp = 0.5 * float((pg.residual(theta + h * dd) ** 2).sum())
        lm = 0.5 * float((pg.residual(theta - h * dd) ** 2).sum())
        fd = (lp - lm) / (2 * h)
        assert abs(grad @ d - fd) <= 1e-6 * max(1.0, abs(fd))
    pg.close()


def test_full_size_ipm_sampled():
    """Full-size IPM-style workload: sampled residual and Jacobian rows of
    every row kind against the oracle, and one step's statistics."""
    inp = workloads.make_inputs_2d("ipm2d")
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pg.set_points_2d(inp["s"], inp["s1"], inp["se"], inp["sval"])
    print(f"\n[gpu 2d] full ipm2d: m={pg.m} P={pg.P}", flush=True)
    theta = inp["theta0"]
    r = pg.residual(dev(theta)).cpu().numpy()
    m = po.m
    e0, d0, b0 = po.n, po.n + 2 * po.n1, po.n + 2 * po.n1 + po.ne
    rows = np.array([0, 1, e0 // 2, e0 - 1, e0, e0 + 1, d0 - 1, d0, b0 - 1, m - 1])
    assert rel(r[rows], po.residual_rows(theta, rows)) < 1e-12
    J, _ = pg.jacobian(dev(theta))
    Jr = J[torch.from_numpy(rows).cuda()].cpu().numpy()
    del J
    torch.cuda.empty_cache()
    Jo = po.jacobian(theta, rows=rows)
    assert rel(Jr, Jo) < 1e-12
    st = pg.eval(dev(theta))
    assert abs(st["half_sq_norm"] - 0.5 * r @ r) <= 1e-12 * (0.5 * r @ r)
    pg.close()
