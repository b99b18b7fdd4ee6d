"""GPU parity of the planned FP64 Gram.

A handle's Gram of order P + 1 runs on a work plan built when the handle is
created. The tiles are dealt evenly to the 8 XCDs. On each XCD, the tiles of
the last round of resident workgroups (two per CU) are split into 2 to 4
K ranges that run side by side. A second launch sums their partial products
in piece order (beta C + piece 0 + piece 1 + ...).

The orders are chosen so that each plan shape runs (256 CUs, 64 resident
workgroups per XCD):
  - P + 1 = 4223 ([1, 63, 63, 1]): 33 tile rows, 561 lower tiles, 70 or 71
    per XCD; the last 6 or 7 on each XCD are split in 4 pieces;
  - P + 1 = 4850 ([1, 48, 48, 48, 1]): 38 tile rows, 741 tiles, 92 or 93 per
    XCD; the last 28 or 29 on each XCD are split in 2;
  - P + 1 = 1154 ([1, 32, 32, 1]): too few 128-tiles for a plan (55), so the
    plan takes 64 x 64 tiles (K step 32): 190 lower tiles, all in the one
    round, each split in 2 pieces;
  - P + 1 = 4548 (2D, [2, 64, 64, 3]) with the rows in three chunks of at
    most 50: G is accumulated chunk by chunk, so the summing launch adds into
    C (beta = 1). A chunk of 50 rows has pieces of 32, 18 and 0 rows (an
    empty piece contributes zeros).

Checks:
  - gn_gram of a random J with m = 300 rows (4 pieces of 80 rows, or 2 of 160
    and 140, the last piece ending in a ragged K chunk; J's row stride is odd
    at order 4223, so its tiles stage through registers, and even at 4850,
    where they copy straight to LDS): every lower entry against the oracle's
    compensated entries, |dG_jk| <= gamma_m |J_j|^T |J_k| (the deterministic
    bound of an m-term FP64 dot product). The upper triangle stays zero.
  - the chunked 2D step: projections w^T v of its normal-equation residual
    v = (J^T J + mu I) d + J^T r on Gaussian directions, from complex-step
    directional derivatives of the oracle residual
    (oracle.gn.projected_normal_residuals), against the bound implied by a
    backward error of 5e-14 (oracle.gn.projected_bound).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import dense
from oracle import gn as ogn
from oracle import profile2d as p2
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def gamma(m):
    u = EPS / 2
    return m * u / (1 - m * u)


@pytest.mark.parametrize("widths", [[1, 63, 63, 1], [1, 48, 48, 48, 1], [1, 32, 32, 1]],
                         ids=["order4223_4pieces", "order4850_2pieces", "order1154_tile64_2pieces"])
def test_planned_gram_every_entry(widths):
    P = workloads.num_params(widths)
    pg = gn.Problem("ccf1d", widths, 0.6057)
    assert pg.P == P
    m = 300
    J = np.random.default_rng(P).standard_normal((m, P + 1))
    print(f"\n[gpu gram plan] order {P + 1}, m = {m}", flush=True)
    G, _ = pg.gram(torch.from_numpy(J).cuda(), None)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy()
    pg.close()
    ref = dense.gram(J)
    A = np.abs(J)
    bound = gamma(m) * (A.T @ A) + 1e-300
    low = np.tril(np.ones((P + 1, P + 1), dtype=bool))
    ratio = np.abs(np.tril(Gg) - np.tril(ref)) / bound
    worst = float(ratio[low].max())
    print(f"[gpu gram plan] worst entry at {worst:.3g} of its bound", flush=True)
    assert worst <= 1.0
    assert not np.any(np.triu(Gg, 1))


def test_planned_gram_chunked_2d_step():
    inp = workloads.make_inputs_2d("bouss2d", n=40, ne=8, nval=16, widths=[2, 64, 64, 3])
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], row_chunk=50)
    pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    assert pg.P == po.P == 4547 and pg.m == po.m and pg.m > 100
    print(f"\n[gpu gram plan] 2D chunked step: m={pg.m} P={pg.P} row chunk 50", flush=True)
    theta = inp["theta0"] + 0.02 * np.random.default_rng(9).standard_normal(po.P)
    mu = 1e-3
    t = torch.from_numpy(theta.copy()).cuda()
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    pg.close()
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, d, mu, k=8, seed=23)
    bound = ogn.projected_bound(pr, mu)
    print(f"[gpu gram plan] projections {np.abs(pr['proj'])} bound {bound}", flush=True)
    assert np.all(np.abs(pr["proj"]) <= bound)
