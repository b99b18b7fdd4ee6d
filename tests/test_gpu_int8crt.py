"""Gram from int8 modular products (precision "int8crt") against
  - the scheme's exact value: every column of J scaled by 2^(b - E_j) and
    rounded to an integer, the integer Gram summed exactly in Python integers
    and scaled back; the kernel must be within 2 ulp of it (the products, sums
    and the reconstruction are exact; only the final conversion rounds);
  - the FP64 oracle Gram J^T J, within the bound of the column rounding
    2^-b (2^E_j S_k + 2^E_k S_j), S_k = sum_i |J_ik|, plus the oracle's own
    FP64 rounding (m + 2) 2^-53 (|J|^T |J|)_jk;
  - the FP64 oracle step, to the same forward-error bar as the FP64 path.
The full-size case (the medium CCF step, 8193 rows, 8514 columns) checks
sampled entries against the exact value and the whole Gram against the FP64
HIP Gram."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import gn as ogn
from oracle import profile1d as p1
from oracle import profile2d as p2
from paper_2509_14185_amd import gn

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53
ULP2 = 2.0 ** -51  # 2 ulp, relative


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def col_exponents(J):
    mx = np.max(np.abs(J), axis=0)
    E = np.zeros(J.shape[1], dtype=np.int64)
    nz = mx > 0
    E[nz] = np.frexp(mx[nz])[1]  # mx = f 2^E, f in [1/2, 1)
    return E, nz


def exact_entries(J, b, pairs):
    """Scheme value of G_jk for each (j, k): integers x = rint(J 2^(b - E)),
    v = sum_i x_ij x_ik in Python integers, scaled by 2^(E_j + E_k - 2b) and
    rounded once (Python's int -> float conversion is correctly rounded)."""
    E, nz = col_exponents(J)
    cols = {}
    for j in {c for pr in pairs for c in pr}:
        x = np.rint(np.ldexp(J[:, j], int(b - E[j]))) if nz[j] else np.zeros(J.shape[0])
        cols[j] = [int(v) for v in x]
    out = []
    for j, k in pairs:
        v = sum(a * c for a, c in zip(cols[j], cols[k]))
        out.append(math.ldexp(float(v), int(E[j] + E[k] - 2 * b)) if v else 0.0)
    return np.array(out)


def int8_problem(widths, n):
    inp = workloads.make_inputs("ccf_small", n=n, m_quad=64, widths=widths)
    pg = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], precision="int8crt")
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    return inp, pg


@pytest.fixture(scope="module")
def handle():
    # P = 321: gn_gram takes up to 322 columns and 512 rows
    inp, pg = int8_problem([1, 16, 16, 1], 511)
    yield pg
    pg.close()


def synthetic_J(m, p, seed):
    """Columns of very different scales, a zero column, a column with a wide
    spread of magnitudes and a constant column."""
    rng = np.random.default_rng(seed)
    J = rng.standard_normal((m, p)) * np.ldexp(1.0, rng.integers(-40, 40, p))[None, :]
    J[:, 3] = 0.0
    J[:, 5] *= np.ldexp(1.0, rng.integers(-30, 1, m))
    J[:, 7] = 0.75
    return J


@pytest.mark.parametrize("m,p", [(300, 70), (512, 322), (1, 9), (129, 200)])
def test_int8_gram_exact(handle, m, p):
    J = synthetic_J(m, p, seed=m + p)
    G, _ = handle.gram(dev(J))
    Gd = G.cpu().numpy()
    b, _ = gn.int8_crt_params(m)
    rng = np.random.default_rng(7)
    pairs = [(j, j) for j in range(p)] + [(j, k) for j in range(p) for k in range(j) if (j + k) % 5 == 0]
    if len(pairs) > 3000:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 3000, replace=False)]
    want = exact_entries(J, b, pairs)
    got = np.array([Gd[j, k] for j, k in pairs])
    err = np.abs(got - want)
    assert np.all(err <= ULP2 * np.abs(want)), f"max rel err {np.max(err / np.maximum(np.abs(want), 1e-300)):.2e}"
    # against the FP64 oracle Gram, within the column-rounding bound
    Go, _ = ogn.gram_and_gradient(J, np.zeros(m))
    E, _ = col_exponents(J)
    S = np.abs(J).sum(axis=0)
    scale = np.ldexp(1.0, E - b)
    bound = scale[:, None] * S[None, :] + S[:, None] * scale[None, :] + (m + 2) * EPS * (np.abs(J).T @ np.abs(J))
    low = np.tril_indices(p)
    d = np.abs(Gd[low] - Go[low])
    assert np.all(d <= bound[low] + ULP2 * np.abs(Go[low]))


def test_int8_gram_strided_with_gradient(handle):
    """J as a view with ldJ > p, and g = J^T r returned with the Gram."""
    m, p, ld = 400, 150, 203
    J = synthetic_J(m, p, seed=9)
    buf = np.full((m, ld), np.nan)
    buf[:, :p] = J
    Jd = dev(buf)[:, :p]
    r = np.random.default_rng(10).standard_normal(m)
    G, g = handle.gram(Jd, dev(r))
    Gd = G.cpu().numpy()
    b, _ = gn.int8_crt_params(m)
    pairs = [(j, k) for j in range(p) for k in range(j + 1) if (3 * j + k) % 7 == 0]
    want = exact_entries(J, b, pairs)
    got = np.array([Gd[j, k] for j, k in pairs])
    assert np.all(np.abs(got - want) <= ULP2 * np.abs(want))
    _, go = ogn.gram_and_gradient(J, r)
    assert rel(g.cpu().numpy(), go) < 1e-12


def test_int8_gram_nonfinite_column(handle):
    m, p = 200, 40
    J = synthetic_J(m, p, seed=3)
    J[17, 9] = np.nan
    J[4, 21] = np.inf
    G, _ = handle.gram(dev(J))
    Gd = np.tril(G.cpu().numpy())
    low = np.tril(np.ones((p, p), dtype=bool))
    bad = np.zeros((p, p), dtype=bool)
    bad[9, :] = bad[:, 9] = bad[21, :] = bad[:, 21] = True
    assert np.all(np.isnan(Gd[bad & low]))
    assert np.all(np.isfinite(Gd[~bad & low]))
    b, _ = gn.int8_crt_params(m)
    pairs = [(j, k) for j in range(p) for k in range(j + 1) if not bad[j, k]]
    want = exact_entries(np.where(np.isfinite(J), J, 0.0), b, pairs)
    got = np.array([Gd[j, k] for j, k in pairs])
    assert np.all(np.abs(got - want) <= ULP2 * np.abs(want))


def test_int8_gram_rejects_oversize(handle):
    J = dev(np.zeros((600, 10)))
    with pytest.raises(gn.GNError):
        handle.gram(J)  # 600 rows > the 512 rows of the workspaces


@pytest.fixture(scope="module", params=["ccf_small", "ccf_ragged"])
def case(request):
    over = {} if request.param == "ccf_small" else dict(n=1000, m_quad=100, widths=[1, 24, 17, 1])
    inp = workloads.make_inputs("ccf_small", **over)
    po = p1.Problem.from_inputs(inp)
    pg = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], precision="int8crt")
    pg.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    yield dict(inp=inp, po=po, pg=pg, theta=inp["theta0"])
    pg.close()


def test_int8_step(case):
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
    print(f"\nint8crt step: |d delta|/|delta| = {ed:.2e} (kappa = {kappa:.1e})")
    assert ed < max(1e-12, 10 * kappa * EPS)
    assert abs(st["half_sq_norm"] - ost["half_sq_norm"]) <= 1e-12 * ost["half_sq_norm"]


def _problem_2d(name, over, row_chunk=0):
    inp = workloads.make_inputs_2d(name, **over)
    pg = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                    precision="int8crt", row_chunk=row_chunk)
    return inp, pg


@pytest.mark.parametrize("name,over", [("ipm2d", dict(n=64, n1=16, ne=8, widths=[2, 12, 12, 1], nval=64)),
                                       ("bouss2d", dict(n=60, ne=8, widths=[2, 10, 10, 3], nval=64))])
def test_int8_step_2d(name, over):
    """2D problems whose J is formed in one chunk: the step against the oracle."""
    inp, pg = _problem_2d(name, over)
    pg.set_points_2d(inp["s"], inp["s1"] if inp["n1"] else None, inp["se"], inp["sval"])
    po = p2.Problem.from_inputs(inp)
    theta, mu = inp["theta0"], 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    ref, ost = ogn.step(po, theta, mu)
    assert ogn.backward_error(ost["G"], mu, ost["g"], d) < 5e-14
    kappa = np.linalg.cond(ost["G"] + mu * np.eye(len(theta)))
    assert rel(d, ref - theta) < max(1e-12, 10 * kappa * EPS)
    pg.close()


@pytest.mark.parametrize("chunk", [37, 100])
def test_int8_step_2d_chunked(chunk):
    """J streamed in row chunks (formed twice: column maxima, then residues
    whose products accumulate modulo m_t): the step against the oracle."""
    inp, pg = _problem_2d("bouss2d", dict(n=70, ne=6, widths=[2, 9, 11, 3], nval=16), row_chunk=chunk)
    pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    po = p2.Problem.from_inputs(inp)
    theta, mu = inp["theta0"], 1e-3
    t = dev(theta)
    st = pg.step(t, mu)
    assert st["rc"] == gn.GN_OK and st["updated"] == 1
    d = t.cpu().numpy() - theta
    ref, ost = ogn.step(po, theta, mu)
    assert ogn.backward_error(ost["G"], mu, ost["g"], d) < 5e-14
    kappa = np.linalg.cond(ost["G"] + mu * np.eye(len(theta)))
    assert rel(d, ref - theta) < max(1e-12, 10 * kappa * EPS)
    pg.close()


def test_int8_two_d_oversize_rejected():
    # 3 x 43700 + 8 + 1 = 131109 rows in one chunk: more than the int8 Gram takes
    inp, pg = _problem_2d("bouss2d", dict(n=43700, ne=8, widths=[2, 4, 3], nval=16))
    with pytest.raises(gn.GNError):
        pg.set_points_2d(inp["s"], None, inp["se"], inp["sval"])
    pg.close()


def test_int8_gram_full_size():
    """Medium CCF step: 8193 rows, 8514 columns of [J | r]."""
    inp = workloads.make_inputs("ccf_medium")
    p64 = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    p64.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    p8 = gn.Problem("ccf1d", inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"], precision="int8crt")
    p8.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    J, r = p64.jacobian(dev(inp["theta0"]))
    Jr = torch.cat([J, r[:, None]], dim=1).contiguous()
    m, p = Jr.shape
    G8, _ = p8.gram(Jr)
    G64, _ = p64.gram(Jr)
    A = Jr.cpu().numpy()
    b, _ = gn.int8_crt_params(m)
    rng = np.random.default_rng(11)
    js = rng.integers(0, p, 48)
    ks = [int(rng.integers(0, j + 1)) for j in js]
    pairs = list(zip(js.tolist(), ks)) + [(p - 1, p - 1), (p - 1, 0), (0, 0)]
    want = exact_entries(A, b, pairs)
    g8 = G8.cpu().numpy()
    got = np.array([g8[j, k] for j, k in pairs])
    assert np.all(np.abs(got - want) <= ULP2 * np.abs(want))
    low = torch.tril(torch.ones(p, p, dtype=torch.bool, device="cuda"))
    diff = torch.where(low, (G8 - G64).abs(), torch.zeros_like(G8))
    # |G8 - G64| against the FP64 Gram's own rounding bound, entry by entry
    absg = torch.where(low, A.shape[0] * EPS * (Jr.abs().T @ Jr.abs()), torch.ones_like(G8))
    worst = float((diff / absg).max())
    print(f"\nfull-size int8crt vs FP64 Gram: max |dG| / (m eps |J|^T|J|) = {worst:.2e}")
    assert worst <= 1.0
    p64.close()
    p8.close()
