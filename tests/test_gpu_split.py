"""Split-precision form (FP32 hi/lo Gram with FP64 accumulation, FP64
residual, gradient, Cholesky and update) against the FP64 oracle.  The error
of each result is printed and held to the bound that FP32 products allow:
  G:      |dG|_F / |G|_F <= 1e-6   (products rounded to FP32, about 6e-8 each)
  r, g:   FP64-exact, <= 1e-12
  delta:  |d delta| / |delta| <= |E| / (lambda_min(G + mu I) - |E|) + 10 kappa eps,
          E the split Gram's measured error ((G~ + mu I) delta~ = -g and (G + mu I)
          delta = -g give d delta = -(G~ + mu I)^-1 E delta)
and the step must still be a descent direction.  From a teacher start (an
exact zero theta* of the residual) the split steps reach the FP64 floor."""
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
    Gm = ost["G"] + mu * np.eye(po.P)
    ev = np.linalg.eigvalsh(Gm)
    kappa = ev[-1] / ev[0]
    # the split Gram's error on the oracle's J (the step's own J agrees with it
    # to FP64 rounding, covered by the 1e-12 |G| term)
    Gs, _ = pg.gram(dev(case["J"]), dev(case["r"]))
    Gs = Gs.cpu().numpy()[: po.P, : po.P]
    Gl = np.tril(Gs) + np.tril(Gs, -1).T
    E = np.linalg.norm(Gl - ost["G"]) + 1e-12 * np.linalg.norm(ost["G"])
    bound = E / (ev[0] - E) + 10 * kappa * np.finfo(np.float64).eps
    ed = rel(d, dref)
    print(f"\nsplit step: |d delta|/|delta| = {ed:.2e}, bound {bound:.2e} (|E|_F = {E:.2e}, "
          f"lambda_min = {ev[0]:.2e}, kappa = {kappa:.1e})")
    assert E < ev[0]
    assert ed <= bound
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


def test_split_teacher_start_reaches_fp64_floor(case):
    """From theta* + 1e-3 v, theta* an exact zero of the residual (source
    f = R[NN_theta*] at the collocation points, c_target = NN_theta*(1)): with
    the damping above the split Gram's FP32 rounding (mu = 1e-6), six split
    steps reach the same floor of |r|^2/2 as six FP64 steps (the residual and
    gradient are FP64, so the fixed point is the same; about 1e-19 from 1e-8);
    with mu = 1e-8 below that rounding the damped split Gram is not positive
    definite, the step is refused (GN_ENOTPD) and theta is left as it was,
    while the FP64 steps still converge."""
    inp = case["inp"]
    po = p1.Problem.from_inputs(inp)
    tstar = case["theta"]
    R, _ = p1.raw_residual(po, tstar)
    f = R.copy()
    NN1, _, _ = p1.mlp_jets(tstar, po.widths, np.ones(1))
    c_target = float(NN1[0])
    po.f, po.c_target = f, c_target
    assert np.linalg.norm(p1.residual_rows(po, tstar)) == 0.0
    v = workloads.perturbation(tstar.size, 3)
    probs = {}
    for prec in ("fp64", "split32"):
        pg = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], c_target, precision=prec)
        pg.set_points(inp["s"], inp["rho"], f, inp["sq"], inp["wq"], inp["sval"])
        probs[prec] = pg
    try:
        traj = {}
        for prec, pg in probs.items():
            t = dev(tstar + 1e-3 * v)
            h = [pg.eval(t)["half_sq_norm"]]
            for _ in range(6):
                assert pg.step(t, 1e-6)["rc"] == gn.GN_OK
                h.append(pg.eval(t)["half_sq_norm"])
            traj[prec] = h
            print(f"\n{prec} from the teacher start, mu 1e-6: " + " ".join(f"{x:.1e}" for x in h))
        a, b = traj["fp64"], traj["split32"]
        assert a[-1] < 1e-9 * a[0] and b[-1] < 1e-9 * b[0]
        assert abs(b[-1] - a[-1]) <= 0.1 * a[-1]
        assert abs(b[1] - a[1]) <= 0.1 * a[1]
        # damping below the split Gram's rounding
        t = dev(tstar + 1e-3 * v)
        t0 = t.clone()
        st = probs["split32"].step(t, 1e-8)
        assert st["rc"] == gn.GN_ENOTPD and torch.equal(t, t0)
        u = dev(tstar + 1e-3 * v)
        for _ in range(3):
            assert probs["fp64"].step(u, 1e-8)["rc"] == gn.GN_OK
        assert probs["fp64"].eval(u)["half_sq_norm"] < 1e-9 * a[0]
    finally:
        for pg in probs.values():
            pg.close()
