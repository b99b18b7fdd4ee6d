"""GPU parity of the 2D steps at sizes where the oracle cannot form the whole
Jacobian:
  - the IPM-style workload at full size (P = 12,737, 98,561 rows): one full
    step;
  - the Boussinesq-type network at its real widths [2, 128, 128, 128, 128, 3]
    (P = 50,307; the jet sweeps take their 4-point tiles at this width) on
    few points, with the rows streamed in several chunks: residual, sampled
    Jacobian columns, validation statistics and one step.

Checks (oracle: oracle/profile2d.py, oracle/gn.py):
  - residual rows: every row, relative 1e-12 (normwise) and
    |dr_i| <= 1e-12 max|r| element-wise;
  - Jacobian: sampled columns (complex step, every row) element by element,
    |dJ_ik| <= 1e-11 max_i |J_ik|, and relative 1e-12 over the sample;
  - the step: projections w^T v of the normal-equation residual
    v = (J^T J + mu I) d + J^T r on Gaussian directions, formed from
    complex-step directional derivatives J w and J d of the oracle residual
    (oracle.gn.projected_normal_residuals), against the bound implied by a
    backward error of 5e-14 (oracle.gn.projected_bound)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile2d as p2
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def check_step_projected(po, theta, d, mu, k, seed):
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, d, mu, k=k, seed=seed)
    bound = ogn.projected_bound(pr, mu)
    print(f"[gpu 2d full] projections {np.abs(pr['proj'])} bound {bound}", flush=True)
    assert np.all(np.abs(pr["proj"]) <= bound)


def test_ipm2d_full_step_projected():
    """One FP64 step of the full IPM-style workload from the Glorot start."""
    inp = workloads.make_inputs_2d("ipm2d")
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    pg.set_points_2d(inp["s"], inp["s1"], inp["se"], inp["sval"])
    print(f"\n[gpu 2d full] ipm2d step: m={pg.m} P={pg.P}", flush=True)
    theta = inp["theta0"]
    mu = inp["mu"]
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    pg.close()
    del t
    torch.cuda.empty_cache()
    check_step_projected(po, theta, d, mu, k=2, seed=21)


BOUSS_REAL = dict(n=40, ne=8, nval=16)  # widths [2, 128, 128, 128, 128, 3]
ROW_CHUNK = 50                           # m = 129 rows: three chunks


@pytest.fixture(scope="module")
def bouss_real():
    inp = workloads.make_inputs_2d("bouss2d", **BOUSS_REAL)
    assert inp["widths"] == [2, 128, 128, 128, 128, 3]
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                    row_chunk=ROW_CHUNK)
    pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    print(f"\n[gpu 2d full] bouss2d real widths: m={pg.m} P={pg.P} row chunk {ROW_CHUNK}", flush=True)
    theta = inp["theta0"] + 0.02 * np.random.default_rng(8).standard_normal(po.P)
    yield dict(inp=inp, po=po, pg=pg, theta=theta)
    pg.close()


def test_bouss_real_widths_residual_and_stats(bouss_real):
    po, pg, theta = bouss_real["po"], bouss_real["pg"], bouss_real["theta"]
    assert pg.m == po.m and pg.P == po.P == 50307
    r = pg.residual(dev(theta)).cpu().numpy()
    ro = po.residual_rows(theta)
    assert rel(r, ro) < 1e-12
    assert np.all(np.abs(r - ro) <= 1e-12 * np.max(np.abs(ro)))
    st = pg.eval(dev(theta))
    assert abs(st["max_abs_R"] - po.train_max(theta)) <= 1e-12 * po.train_max(theta)
    assert abs(st["max_abs_R_val"] - po.validation_max(theta)) <= 1e-12 * po.validation_max(theta)


def sampled_columns(widths, rng, per_block=6):
    """Columns from every weight and bias block (first, last and random
    entries of each), so every layer's part of the reverse sweep is seen."""
    cols, o = [], 0
    for a, b in zip(widths[:-1], widths[1:]):
        for size in (a * b, b):
            pick = {o, o + size - 1}
            pick.update(int(x) for x in o + rng.integers(0, size, per_block))
            cols.extend(sorted(pick))
            o += size
    return np.array(cols)


def test_bouss_real_widths_jacobian_columns(bouss_real):
    po, pg, theta = bouss_real["po"], bouss_real["pg"], bouss_real["theta"]
    cols = sampled_columns(po.widths, np.random.default_rng(13))
    J, r = pg.jacobian(dev(theta))
    Jg = J[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    del J
    torch.cuda.empty_cache()
    Jo = po.jacobian(theta, cols=cols)
    assert rel(Jg, Jo) < 1e-12
    scale = np.max(np.abs(Jo), axis=0)
    bad = np.abs(Jg - Jo) > 1e-11 * scale[None, :]
    assert not bad.any(), f"{bad.sum()} entries off, columns {np.unique(cols[np.nonzero(bad)[1]])}"
    assert rel(r.cpu().numpy(), po.residual_rows(theta)) < 1e-12


def test_bouss_real_widths_chunked_step(bouss_real):
    """FP64 step with the Gram accumulated over three row chunks."""
    po, pg, theta = bouss_real["po"], bouss_real["pg"], bouss_real["theta"]
    mu = 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1 and st["chol_info"] == 0
    d = t.cpu().numpy() - theta
    r = po.residual_rows(theta)
    assert abs(st["half_sq_norm"] - 0.5 * r @ r) <= 1e-12 * (0.5 * r @ r)
    check_step_projected(po, theta, d, mu, k=8, seed=22)


U32 = 2.0 ** -24


@pytest.mark.parametrize("precision", ["fp64", "split32"])
def test_bouss_real_widths_gram_entries(bouss_real, precision):
    """Gram entries of the sampled columns (every pair, diagonal included)
    against the oracle's compensated products of its own J columns.  With
    D = J_gpu - J_oracle on those columns (checked separately),
    |dG_jk| <= c (|J|^T |J|)_jk + (|D|^T |J| + |J|^T |D| + |D|^T |D|)_jk,
    c = gamma_m (FP64) or 40 u32 (the split form: FP32 sums of 32-row chunks
    of hi/lo products): the Gram's own rounding plus what the difference of
    its input carries.  The observed ratio to the bound is printed."""
    from oracle import dense

    inp, po, theta = bouss_real["inp"], bouss_real["po"], bouss_real["theta"]
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], precision=precision)
    pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    cols = sampled_columns(po.widths, np.random.default_rng(14))
    J, _ = pg.jacobian(dev(theta), with_r=False)
    ci = torch.from_numpy(cols).cuda()
    Jg = J[:, ci].cpu().numpy()
    G, _ = pg.gram(J)
    Gs = G[ci][:, ci].cpu().numpy()
    del G, J
    pg.close()
    torch.cuda.empty_cache()
    Jo = po.jacobian(theta, cols=cols)
    Go = dense.gram(Jo)
    A, D = np.abs(Jo), np.abs(Jg - Jo)
    m = Jo.shape[0]
    c = m * (EPS / 2) / (1 - m * EPS / 2) if precision == "fp64" else 40 * U32
    bound = c * (A.T @ A) + D.T @ A + A.T @ D + D.T @ D
    low = cols[:, None] >= cols[None, :]
    ratio = (np.abs(Gs - Go) / bound)[low]
    print(f"[gpu 2d full] {precision} Gram entries: max |dG| / bound = {ratio.max():.3e}; "
          f"max |dG| / (|J|^T |J|) = {(np.abs(Gs - Go) / (A.T @ A))[low].max():.3e}", flush=True)
    assert ratio.max() <= 1.0


def test_bouss_real_widths_split_chunked_step():
    """Split-precision step with the Gram accumulated over three row chunks:
    the projections of the normal-equation residual against the bound of a
    backward error of 1e-5 (the split Gram's own relative error is about
    32 u32 = 2e-6 of |J|^T |J|)."""
    inp = workloads.make_inputs_2d("bouss2d", **BOUSS_REAL)
    po = p2.Problem.from_inputs(inp)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                    precision="split32", row_chunk=ROW_CHUNK)
    pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    theta = inp["theta0"] + 0.02 * np.random.default_rng(8).standard_normal(po.P)
    mu = 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    pg.close()
    torch.cuda.empty_cache()
    pr = ogn.projected_normal_residuals(po.residual_rows, theta, d, mu, k=8, seed=23)
    fp64_bound = ogn.projected_bound(pr, mu)
    print(f"[gpu 2d full] split step: max |w^T v| / (5e-14 bound) = {np.max(np.abs(pr['proj']) / fp64_bound):.3e}",
          flush=True)
    assert np.all(np.abs(pr["proj"]) <= ogn.projected_bound(pr, mu, b=1e-5))
