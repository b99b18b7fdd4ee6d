"""GPU parity of the batched step (gn_step_batched) against the CPU FP64
oracle and against the single-instance gn_step.

Instances differ in blow-up rate lambda, point count and seed (batched CCF
workload).  Tolerances as for the single step: backward error of the solve
<= 5e-14, forward error <= max(1e-12, 10 kappa eps), statistics relative
1e-12; batched versus single-instance steps agree to 1e-12 (same kernels,
summation order may differ only in the reductions)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def make_problem(inp):
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    return pg


def check_against_oracle(inp, theta0, theta1, st, mu):
    po = p1.Problem.from_inputs(inp)
    ref, ost = ogn.step(po, theta0, mu)
    d, dref = theta1 - theta0, ref - theta0
    G, g = ost["G"], ost["g"]
    assert ogn.backward_error(G, mu, g, d) < 5e-14
    kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
    assert rel(d, dref) < max(1e-12, 10 * kappa * EPS)
    assert abs(st["half_sq_norm"] - ost["half_sq_norm"]) <= 1e-12 * ost["half_sq_norm"]
    gd = float(g @ dref)
    assert st["grad_dot_delta"] < 0 and abs(st["grad_dot_delta"] - gd) <= 1e-10 * abs(gd)
    R, _ = p1.raw_residual(po, theta0)
    assert abs(st["max_abs_R"] - np.max(np.abs(R))) <= 1e-12 * np.max(np.abs(R))
    assert abs(st["max_abs_R_val"] - p1.validation_max(po, theta0)) <= 1e-12 * p1.validation_max(po, theta0)


@pytest.fixture(scope="module", params=["w20", "w32"])
def small(request):
    # w20: P = 481, the bordered order 482 spans four 128-wide panels with a
    # ragged tail; w32: P = 1153, the bordered order 1154 = 9 x 128 + 2, whose
    # last two Gram rows go to the batched product of 32-row tiles
    widths, n_range = ([1, 20, 20, 1], (200, 900)) if request.param == "w20" else ([1, 32, 32, 1], (200, 600))
    print(f"\n[gpu batch] small batch: 5 instances, widths {widths}, n in {list(n_range)}", flush=True)
    inps = workloads.make_batched_inputs(instances=5, n_range=n_range, m_quad=64, widths=widths, seed=9)
    pgs = [make_problem(x) for x in inps]
    b = gn.Batch(pgs)
    yield inps, pgs, b
    b.close()
    for p in pgs:
        p.close()


def test_batched_step_matches_oracle(small):
    inps, pgs, b = small
    mu = 1e-3
    ts = [dev(x["theta0"]) for x in inps]
    sts = b.step(ts, mu)
    for inp, t, st in zip(inps, ts, sts):
        assert st["rc"] == gn.GN_OK and st["updated"] == 1 and st["chol_info"] == 0
        check_against_oracle(inp, inp["theta0"], t.cpu().numpy(), st, mu)


def test_batched_matches_single(small):
    """Two batched steps against two single steps per instance.  The first
    step's residual statistics come from the same kernels at the same theta
    (equal to 1e-14); its model value and g^T delta come from Grams, factors
    and solves with other summation orders (compared on the scale of r^T r,
    of which the bordered factor's corner is a difference; the oracle check
    takes 1e-8 r^T r).  The second step starts from iterates that differ by
    the rounding of the first update, so its statistics are compared at
    1e-10; the sums of the two updates agree to 20 kappa eps (each update
    within 10 kappa eps of the exact one, as in the oracle check)."""
    inps, pgs, b = small
    mu = 1e-3
    ts = [dev(x["theta0"]) for x in inps]
    sts1 = b.step(ts, mu)
    sts2 = b.step(ts, mu)  # second step: new iterate, same descriptors
    for inp, pg, t, st1, st2 in zip(inps, pgs, ts, sts1, sts2):
        u = dev(inp["theta0"])
        s1 = pg.step(u, mu)
        s2 = pg.step(u, mu)
        # the two updates, each within 10 kappa eps of the exact one (the
        # oracle check's bound; kappa of G + mu I at the start)
        G = ogn.step(p1.Problem.from_inputs(inp), inp["theta0"], mu)[1]["G"]
        kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
        d_b, d_s = t.cpu().numpy() - inp["theta0"], u.cpu().numpy() - inp["theta0"]
        assert rel(d_b, d_s) < max(1e-12, 20 * kappa * EPS)
        rr = 2 * s1["half_sq_norm"]
        for k in ("half_sq_norm", "max_abs_R", "max_abs_R_val"):
            assert abs(st1[k] - s1[k]) <= 1e-14 * abs(s1[k])
            assert abs(st2[k] - s2[k]) <= 1e-10 * abs(s2[k])
        for k in ("model_sq_norm", "grad_dot_delta"):
            assert abs(st1[k] - s1[k]) <= 1e-12 * rr
            assert abs(st2[k] - s2[k]) <= 1e-10 * 2 * s2["half_sq_norm"]


def test_batched_new_parameter_buffers_and_determinism(small):
    inps, pgs, b = small
    a = [dev(x["theta0"]) for x in inps]
    c = [dev(x["theta0"]) for x in inps]
    b.step(a, 1e-3, stats=False)
    b.step(c, 1e-3, stats=False)
    torch.cuda.synchronize()
    for x, y in zip(a, c):
        assert torch.equal(x, y)


def test_batched_failure_is_isolated(small):
    inps, pgs, b = small
    good = [dev(x["theta0"]) for x in inps]
    b.step(good, 1e-3)
    bad_np = inps[2]["theta0"].copy()
    bad_np[5] = np.nan
    ts = [dev(x["theta0"]) for x in inps]
    ts[2] = dev(bad_np)
    sts = b.step(ts, 1e-3)
    assert sts[2]["rc"] == gn.GN_ENONFINITE and sts[2]["updated"] == 0
    got = ts[2].cpu().numpy()
    keep = ~np.isnan(bad_np)
    assert np.array_equal(got[keep], bad_np[keep])
    for i in (0, 1, 3, 4):
        assert sts[i]["rc"] == gn.GN_OK and sts[i]["updated"] == 1
        assert torch.equal(ts[i], good[i])


def test_batch_argument_checks(small):
    inps, pgs, b = small
    with pytest.raises(ValueError):
        b.step([dev(inps[0]["theta0"])], 1e-3)
    with pytest.raises(gn.GNError) as e:
        b.step([dev(x["theta0"]) for x in inps], -1.0)
    assert e.value.status == gn.GN_EINVAL
    # mixed parameter counts are rejected
    other = gn.Problem("ccf1d", [1, 8, 1], 0.5)
    other.set_points(inps[0]["s"], None, None, inps[0]["sq"], inps[0]["wq"], None)
    with pytest.raises(gn.GNError) as e:
        gn.Batch([pgs[0], other])
    assert e.value.status == gn.GN_EINVAL
    other.close()


def test_batch_mixed_equations():
    """A Burgers instance (no Hilbert coupling) beside CCF instances."""
    inps = workloads.make_batched_inputs(instances=3, n_range=(150, 400), m_quad=48, widths=[1, 12, 12, 1], seed=5)
    inps[1]["equation"] = "burgers1d"
    inps[1]["c_target"] = -1.0
    pgs = []
    for x in inps:
        ccf = x["equation"] == "ccf1d"
        p = gn.Problem(x["equation"], x["widths"], x["lam"], x["c_norm"], x["c_target"])
        p.set_points(x["s"], x["rho"], x["f"], x["sq"] if ccf else None, x["wq"] if ccf else None, x["sval"])
        pgs.append(p)
    b = gn.Batch(pgs)
    ts = [dev(x["theta0"]) for x in inps]
    sts = b.step(ts, 1e-3)
    for x, t, st in zip(inps, ts, sts):
        assert st["rc"] == gn.GN_OK
        po = p1.Problem.from_inputs(x, equation=x["equation"])
        ref, ost = ogn.step(po, x["theta0"], 1e-3)
        d, dref = t.cpu().numpy() - x["theta0"], ref - x["theta0"]
        assert ogn.backward_error(ost["G"], 1e-3, ost["g"], d) < 5e-14
        kappa = np.linalg.cond(ost["G"] + 1e-3 * np.eye(ost["G"].shape[0]))
        assert rel(d, dref) < max(1e-12, 10 * kappa * EPS)
    b.close()
    for p in pgs:
        p.close()


def test_batch_stale_after_set_points():
    inps = workloads.make_batched_inputs(instances=2, n_range=(100, 200), m_quad=32, widths=[1, 8, 8, 1], seed=3)
    pgs = [make_problem(x) for x in inps]
    b = gn.Batch(pgs)
    ts = [dev(x["theta0"]) for x in inps]
    assert all(s["rc"] == gn.GN_OK for s in b.step(ts, 1e-3))
    x = inps[1]
    pgs[1].set_points(x["s"], x["rho"], x["f"], x["sq"], x["wq"], x["sval"])
    with pytest.raises(gn.GNError) as e:
        b.step(ts, 1e-3)
    assert e.value.status == gn.GN_ESTATE
    b.close()
    for p in pgs:
        p.close()


def test_full_batched_workload_sampled():
    """64 instances at full size: every instance against its own single-
    instance step; the smallest instance against the oracle.

    The single-instance Gram of order 1154 runs on a work plan of 64 x 64
    tiles whose K range is split in two pieces, while the batched Gram sums
    each tile over the whole K range: the two steps add in different orders,
    so they agree to what their backward errors allow, not bitwise. If both
    have normwise backward error at most eta = 5e-14 (the level the oracle
    check asserts), then (G + mu I)(d1 - d2) is the difference of their
    residuals, and with |(G + mu I)^-1| <= 1/mu (G is semidefinite)
        |d1 - d2| <= eta / mu * ((|J|_F^2 + mu sqrt(P)) (|d1| + |d2|) + 2 |J|_F |r|)."""
    inps = workloads.make_batched_inputs()
    print(f"\n[gpu batch] full batch: {len(inps)} instances, N total {sum(x['n'] for x in inps)}", flush=True)
    pgs = [make_problem(x) for x in inps]
    b = gn.Batch(pgs)
    mu = inps[0]["mu"]
    ts = [dev(x["theta0"]) for x in inps]
    sts = b.step(ts, mu)
    assert all(s["rc"] == gn.GN_OK and s["updated"] == 1 for s in sts)
    eta = 5e-14
    for inp, pg, t in zip(inps, pgs, ts):
        u = dev(inp["theta0"])
        J, r = pg.jacobian(u)
        nJ, nr = torch.linalg.norm(J).item(), torch.linalg.norm(r).item()
        del J, r
        pg.step(u, mu)
        d1, d2 = t.cpu().numpy() - inp["theta0"], u.cpu().numpy() - inp["theta0"]
        n1, n2 = np.linalg.norm(d1), np.linalg.norm(d2)
        bound = eta / mu * ((nJ * nJ + mu * np.sqrt(pg.P)) * (n1 + n2) + 2 * nJ * nr)
        assert np.linalg.norm(d1 - d2) <= bound
    k = int(np.argmin([x["n"] for x in inps]))
    print(f"[gpu batch] oracle check of instance {k} (n={inps[k]['n']})", flush=True)
    check_against_oracle(inps[k], inps[k]["theta0"], ts[k].cpu().numpy(), sts[k], mu)
    b.close()
    for p in pgs:
        p.close()
