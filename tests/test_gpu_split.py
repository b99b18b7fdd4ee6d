"""Split-precision form (FP32 hi/lo Gram with FP64 accumulation, FP64
residual, gradient, Cholesky and update) against the FP64 oracle.  The error
of each result is printed and held to the bound that FP32 products allow:
  G:      |dG|_F / |G|_F <= 1e-6   (products rounded to FP32, about 6e-8 each)
  r, g:   FP64-exact, <= 1e-12
  delta:  |d delta| / |delta| <= 1e-6 * kappa(G + mu I) (inexact Newton step)
and the step must still be a descent direction."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module", params=["ccf_small", "ccf_ragged"])
def case(request):
    over = {} if request.param == "ccf_small" else dict(n=1000, m_quad=100, widths=[1, 24, 17, 1])
    inp = workloads.make_inputs("ccf_small", **over)
    po = p1.Problem.from_inputs(inp)
    pg = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], precision="split32")
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    theta = inp["theta0"]
    r = p1.residual_rows(po, theta)
    J = p1.jacobian(po, theta)
    G, g = ogn.gram_and_gradient(J, r)
    yield dict(inp=inp, po=po, pg=pg, theta=theta, r=r, J=J, G=G, g=g)
    pg.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def test_split_gram_error(case):
    G, g = case["pg"].gram(dev(case["J"]), dev(case["r"]))
    eg = rel(np.tril(G.cpu().numpy()), np.tril(case["G"]))
    print(f"\nsplit Gram: |dG|/|G| = {eg:.2e}")
    assert eg < 1e-6
    assert rel(g.cpu().numpy(), case["g"]) < 1e-12


def test_split_step(case):
    po, pg, theta = case["po"], case["pg"], case["theta"]
    mu = 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    ref, ost = ogn.step(po, theta, mu)
    dref = ref - theta
    kappa = np.linalg.cond(ost["G"] + mu * np.eye(po.P))
    ed = rel(d, dref)
    print(f"\nsplit step: |d delta|/|delta| = {ed:.2e} (kappa = {kappa:.1e})")
    assert ed < 1e-6 * kappa
    assert abs(st["half_sq_norm"] - ost["half_sq_norm"]) <= 1e-12 * ost["half_sq_norm"]
    assert st["grad_dot_delta"] < 0 and float(ost["g"] @ d) < 0


def test_split_reaches_fp64_residual(case):
    """Inexact Newton with an FP64 residual: same fixed point, so after a few
    steps the validation max-norm matches the FP64 trajectory closely."""
    inp, theta = case["inp"], case["theta"]
    p64 = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    p64.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    a, b = dev(theta), dev(theta)
    for _ in range(5):
        p64.step(a, 1e-3)
        case["pg"].step(b, 1e-3)
    va, vb = p64.eval(a)["half_sq_norm"], case["pg"].eval(b)["half_sq_norm"]
    print(f"\nafter 5 steps: FP64 |r|^2/2 = {va:.6e}, split {vb:.6e}")
    assert abs(va - vb) <= 1e-3 * va
    p64.close()
