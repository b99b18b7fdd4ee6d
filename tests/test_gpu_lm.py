"""GPU parity of the Levenberg-Marquardt step (gn_step_lm) against the
oracle's lm_step on identical seeded inputs: each step starts both sides from
the oracle's theta and damping.  Compared: the outcome (accepted or
rejected), the number of factorisations, the returned damping (decided in
FP64 on both sides from the gain ratio; a ratio within 1e-6 of a threshold
would make the decision rounding-dependent and is reported instead), the gain
ratio (relative 1e-6: at tiny damping the trial update carries the condition
number of G + mu I), theta (forward error <= max(1e-12, 10 kappa eps)) and
the objective at the returned point (relative 1e-10).  Cases: 1D CCF and
Burgers with many rejected trials (the retries factor the saved copy of G
again), a case rejected until max_tries, an exactly singular G (a dead
neuron) with mu = 0 first, a 2D stand-in, and the argument checks."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1
from oracle import profile2d as p2
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps

CASES_1D = {
    "ccf_small": ("ccf_small", {}, "ccf1d"),
    "ccf_ragged": ("ccf_small", dict(n=1000, m_quad=100, widths=[1, 24, 17, 1]), "ccf1d"),
    "burgers": ("ccf_small", dict(n=777, widths=[1, 16, 16, 1]), "burgers1d"),
}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def build_1d(key):
    name, over, eq = CASES_1D[key]
    inp = workloads.make_inputs(name, **over)
    if eq == "burgers1d":
        inp["c_target"] = -1.0
    po = p1.Problem.from_inputs(inp, equation=eq)
    pg = gn.Problem(eq, inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    ccf = eq == "ccf1d"
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"] if ccf else None, inp["wq"] if ccf else None,
                  inp["sval"])
    return inp, po, pg


def near_threshold(rho, kw):
    o = dict(ogn.LM_DEFAULTS)
    o.update(kw)
    return any(abs(rho - t) < 1e-6 for t in (0.0, o["rho_lo"], o["rho_hi"]))


def compare(po, pg, theta, mu, **kw):
    """One LM step on both sides from the same theta and mu; returns the oracle's result."""
    ref, out = ogn.lm_step(po, theta, mu, **kw)
    t = dev(theta)
    st = pg.step_lm(t, mu, **kw)
    got = t.cpu().numpy()
    print(f"  mu {mu:.3g}: oracle {out['status']} tries {out['tries']} rho {out['rho']:.6g}; "
          f"gpu rc {st['rc']} tries {st['tries']} rho {st['rho']:.6g}", flush=True)
    assert st["tries"] == out["tries"]
    assert (st["rc"] == gn.GN_OK) == (out["status"] == "ok")
    if out["status"] == "ok":
        assert st["rho"] == pytest.approx(out["rho"], rel=1e-6, abs=1e-9)
        if not near_threshold(out["rho"], kw):
            assert st["mu"] == pytest.approx(out["mu"], rel=1e-15)
        assert st["half_sq_norm_new"] == pytest.approx(out["half_sq_norm_new"], rel=1e-10)
        # forward error of the accepted update
        J = ogn._jacobian(po, theta)
        mu_acc = out["mus"][-1]
        kappa = np.linalg.cond(J.T @ J + mu_acc * np.eye(J.shape[1]))
        d, dref = got - theta, ref - theta
        assert np.linalg.norm(d - dref) <= max(1e-12, 10 * kappa * EPS) * np.linalg.norm(dref)
    else:
        assert st["rc"] == gn.GN_EREJECTED
        assert np.array_equal(got, theta)
        assert st["mu"] == pytest.approx(out["mu"], rel=1e-15)
        assert st["half_sq_norm_new"] == pytest.approx(out["half_sq_norm"], rel=1e-12)
    assert st["half_sq_norm"] == pytest.approx(out["half_sq_norm"], rel=1e-12)
    return ref, out


@pytest.mark.parametrize("key", list(CASES_1D))
def test_lm_trajectory_1d(key):
    print(f"\n[gpu lm] {key}", flush=True)
    inp, po, pg = build_1d(key)
    theta, mu = inp["theta0"], 1e-9
    for k in range(3):
        theta_next, out = compare(po, pg, theta, mu, up=10.0)
        if k == 0:
            assert out["tries"] > 1      # the retry path ran
        theta, mu = theta_next, out["mu"]
    pg.close()


def test_lm_rejected_until_max_tries():
    print("\n[gpu lm] ccf_ragged rejected", flush=True)
    inp, po, pg = build_1d("ccf_ragged")
    ref, out = compare(po, pg, inp["theta0"], 1e-9, up=2.0, max_tries=6)
    assert out["status"] == "rejected" and out["tries"] == 6
    pg.close()


def test_lm_rejection_at_mu_max_stops():
    inp, po, pg = build_1d("ccf_small")
    ref, out = compare(po, pg, inp["theta0"], 1e-9, up=10.0, mu_max=1e-7)
    assert out["status"] == "rejected" and out["mus"] == pytest.approx([1e-9, 1e-8, 1e-7])
    pg.close()


def test_lm_singular_gram_retries_with_mu_min():
    print("\n[gpu lm] dead neuron", flush=True)
    inp, po, pg = build_1d("burgers")
    theta = inp["theta0"].copy()
    # widths [1, 16, 16, 1]: W1 (16), b1 (16), W2 (16 x 16), b2 (16), W3 (16), b3 (1)
    k = 5
    w2 = 32
    theta[w2 + 16 * k: w2 + 16 * (k + 1)] = 0.0     # incoming weights of neuron k, layer 2
    theta[w2 + 256 + k] = 0.0                       # its bias
    theta[w2 + 256 + 16 + k] = 0.0                  # its outgoing weight
    # with mu = 0 the factorisation fails on both sides (at the zero column
    # w2 + 16 k + 1 at the latest; rounding may stop it earlier), then mu_min
    ref, out = compare(po, pg, theta, 0.0, mu_min=1e-3)
    assert 0 < out["infos"][0] <= w2 + 16 * k + 1 and out["infos"][-1] == 0
    assert out["mus"][:2] == [0.0, 1e-3]
    pg.close()


def test_lm_2d():
    print("\n[gpu lm] ipm2d small", flush=True)
    inp = workloads.make_inputs_2d("ipm2d", n=64, n1=16, ne=8, widths=[2, 12, 12, 1], nval=64)
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pg.set_points_2d(inp["s"], inp["s1"], inp["se"], inp["sval"])
    theta, mu = inp["theta0"], 1e-6
    for k in range(2):
        theta, out = compare(po, pg, theta, mu, up=10.0)
        mu = out["mu"]
    pg.close()


def test_lm_argument_checks():
    inp, po, pg = build_1d("ccf_small")
    t = dev(inp["theta0"])
    for bad in (dict(up=1.0), dict(down=0.5), dict(mu_min=0.0), dict(rho_lo=0.8, rho_hi=0.5), dict(max_tries=0),
                dict(mu_max=1e-20)):
        with pytest.raises(gn.GNError) as e:
            pg.step_lm(t, 1e-3, **bad)
        assert e.value.status == gn.GN_EINVAL
    assert np.array_equal(t.cpu().numpy(), inp["theta0"])
    pg.close()
