"""GPU parity of the damped solve at an order with many outer panels of the
blocked Cholesky (n = 2100: five 512-wide outer panels, the last one ragged), so
that every part of the schedule runs: the side stream's trailing update in
row chunks and in two K halves, the panel-after-next columns first, the
joins.  Against the oracle: the normwise backward error of the solve
(oracle/gn.backward_error) <= 5e-14, the update against oracle/gn
damped_solve to max(1e-12, 10 kappa eps), the factor against the oracle's
textbook Cholesky (oracle/dense.c) to max(1e-12, 10 sqrt(kappa) eps).  G is
the Gram of a seeded random J (2500 x 2100) with column scales spread over
four decades."""
import numpy as np
import pytest
import torch

import workloads
from oracle import dense
from oracle import gn as ogn
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def big():
    print("\n[gpu solve panels] n = 2100", flush=True)
    rng = np.random.default_rng(17)
    n, m = 2100, 2500
    J = rng.standard_normal((m, n)) * np.logspace(0, -4, n)[None, :]
    G = J.T @ J
    g = rng.standard_normal(n)
    # a handle whose workspace holds an order-2100 system (any 1D problem with P >= 2100)
    inp = workloads.make_inputs("ccf_medium")
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    yield G, g, pg
    pg.close()


@pytest.mark.parametrize("mu", [1e-6, 1e-2])
def test_solve_many_panels(big, mu):
    G, g, pg = big
    Gd = torch.from_numpy(np.ascontiguousarray(np.tril(G))).cuda()
    delta, info = pg.solve(Gd, mu, torch.from_numpy(g).cuda())
    assert info == 0
    d = delta.cpu().numpy()
    assert ogn.backward_error(G, mu, g, d) < 5e-14
    ref, oinfo = ogn.damped_solve(G, g, mu)
    assert oinfo == 0
    kappa = np.linalg.cond(G + mu * np.eye(G.shape[0]))
    assert rel(d, ref) < max(1e-12, 10 * kappa * EPS)
    L = np.tril(Gd.cpu().numpy())
    Lo, _ = dense.cholesky(G + mu * np.eye(G.shape[0]))
    assert rel(L, Lo) < max(1e-12, 10 * np.sqrt(kappa) * EPS)
