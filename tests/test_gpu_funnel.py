"""GPU parity of funnel inference (gn_funnel_residual and the driver
paper_2509_14185_amd.funnel) against the oracle (oracle/funnel.py on the
oracle's validation residual) on identical seeded inputs.  The proxy is a
selection: the GPU's value must be the oracle's residual at the point the GPU
picked (relative 1e-12 of max |R|) and of largest magnitude in the
neighbourhood (to the same tolerance, so near-ties may pick either point).
Cases: CCF and the local variant, several neighbourhoods (one point, about
200, all), the argument checks, and three outer iterations of the driver
whose lam sequence must follow the oracle's secant update of the measured
proxies."""
import numpy as np
import pytest
import torch

import workloads
from oracle import funnel as fo
from oracle import profile1d as p1
from paper_2509_14185_amd import funnel as fn
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def setup(eq, lam=None):
    inp = workloads.make_inputs("ccf_small", n=300, m_quad=64, widths=[1, 12, 10, 1])
    if eq == p1.BURGERS:
        inp["c_target"] = -1.0
    if lam is not None:
        inp["lam"] = lam
    return inp


def gpu_problem(eq, inp):
    ccf = eq == p1.CCF
    pg = gn.Problem(eq, inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"] if ccf else None, inp["wq"] if ccf else None,
                  inp["sval"])
    return pg


def oracle_val_residual(eq, inp, theta):
    base_v = p1.Problem(eq, inp["widths"], inp["lam"], inp["sval"], sq=inp["sq"], wq=inp["wq"])
    R, _ = p1.raw_residual(base_v, theta)
    return R, base_v.y


def check_proxy(r, y_at, R, y, y_max):
    inside = y <= y_max
    top = np.max(np.abs(R[inside]))
    tol = 1e-12 * max(top, 1e-300)
    j = int(np.argmin(np.abs(y - y_at)))
    assert inside[j] and abs(y[j] - y_at) <= 1e-14 * max(1.0, y_at)
    assert abs(R[j] - r) <= tol
    assert abs(r) >= top - tol
    ro, yo = fo.proxy(R, y, y_max)
    second = np.sort(np.abs(R[inside]))[-2] if inside.sum() > 1 else -np.inf
    if top - second > 2 * tol:  # a unique largest magnitude: the same point on both sides
        assert yo == y[j]
        assert r == pytest.approx(ro, rel=1e-12)


@pytest.mark.parametrize("eq", [p1.CCF, p1.BURGERS])
def test_proxy_matches_oracle(eq):
    print(f"\n[gpu funnel] proxy {eq}", flush=True)
    inp = setup(eq)
    pg = gpu_problem(eq, inp)
    theta = inp["theta0"] + 0.05 * np.random.default_rng(3).standard_normal(pg.P)
    R, y = oracle_val_residual(eq, inp, theta)
    t = dev(theta)
    for y_max in (0.0, 0.05, 1.0, 1e300):
        r, y_at = pg.funnel_residual(t, y_max)
        check_proxy(r, y_at, R, y, y_max)
    pg.close()


def test_argument_checks():
    inp = setup(p1.CCF)
    pg = gpu_problem(p1.CCF, inp)
    t = dev(inp["theta0"])
    with pytest.raises(gn.GNError) as e:
        pg.funnel_residual(t, -1.0)          # no validation point with y <= -1
    assert e.value.status == gn.GN_ESTATE
    with pytest.raises(gn.GNError) as e:
        pg.funnel_residual(t, float("nan"))
    assert e.value.status == gn.GN_EINVAL
    pg.close()
    pn = gn.Problem(p1.CCF, inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pn.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], None)   # no validation grid
    with pytest.raises(gn.GNError) as e:
        pn.funnel_residual(t, 1.0)
    assert e.value.status == gn.GN_ESTATE
    pn.close()


def test_driver_follows_the_secant():
    print("\n[gpu funnel] driver", flush=True)
    eq = p1.CCF
    inp0 = setup(eq)
    lam0, dlam, mu, y_max = 0.58, 0.01, 1e-3, 1.0
    theta = dev(inp0["theta0"])
    snaps = []

    def make(lam):
        return gpu_problem(eq, setup(eq, lam))

    def on_iter(n, lam, r, y):
        snaps.append(theta.cpu().numpy().copy())

    lams, rs, ys = fn.funnel_inference(make, theta, lam0, dlam, 3, 2, mu, y_max, on_iter=on_iter)
    assert lams[0] == lam0 and lams[1] == lam0 + dlam
    assert lams[2] == pytest.approx(fo.secant_next(lams[:2], rs[:2], dlam), rel=1e-15)
    for lam, r, y_at, th in zip(lams, rs, ys, snaps):
        R, y = oracle_val_residual(eq, setup(eq, lam), th)
        check_proxy(r, y_at, R, y, y_max)
    assert fn.next_lambda([0.5, 0.6], [0.2, 0.2], 0.01) == 0.6
