"""Host-side parameters of the int8 modular Gram (no GPU): the moduli are
pairwise coprime and fit int8 residues, the kept bits b make every integer
Gram entry |v| <= m 2^(2b) fall below M / 4, and the reconstruction
v = sum_t y_t W_t - Q M with Q = rint(sum_t y_t fl(W_t / M)) recovers v from its
residues (checked here in Python integers, independently of the kernels)."""
import math
import random

import pytest

from paper_2509_14185_amd import gn


def params(m):
    return gn.int8_crt_params(m)


def test_moduli_coprime_and_small():
    _, mods = params(8193)
    assert len(mods) == 16
    for i, a in enumerate(mods):
        assert 2 <= a <= 256
        for b in mods[i + 1:]:
            assert math.gcd(a, b) == 1
    M = math.prod(mods)
    # W_t < M fit four 40-bit limbs, and 16 residues (< 256) times a limb sum
    # below 2^53: the limb sums are exact in FP64
    assert M < 2 ** 160
    assert 16 * 255 * (2 ** 40 - 1) < 2 ** 53


@pytest.mark.parametrize("m", [1, 2, 100, 1000, 8193, 65536, 130944, 130945, 786689, 2 ** 30])
def test_bits_bound(m):
    b, mods = params(m)
    M = math.prod(mods)
    assert m * 2 ** (2 * b) < M // 4
    assert b <= 58
    if b < 58:  # b is the largest such value (up to the one bit of margin)
        assert m * 2 ** (2 * (b + 2)) >= M // 4


def test_medium_step_bits():
    # 8193 rows of the medium CCF step keep 54 bits per column
    assert params(8193)[0] == 54


def test_streamed_total_rows_bits():
    # the Boussinesq-type step streams 786,689 rows in 24 chunks; its columns
    # keep 51 bits (b from the total row count, not a chunk's)
    assert params(786689)[0] == 51
    assert params(32768)[0] > params(786689)[0]


@pytest.mark.parametrize("m", [0, -1, 2 ** 40 + 1])
def test_rejects(m):
    with pytest.raises(gn.GNError):
        params(m)


def balanced(x, mt):
    r = x % mt
    return r - mt if r >= (mt + 1) // 2 else r


def test_reconstruction_formula():
    """Residues of exact integer Grams of random int vectors reproduce the
    sum (the arithmetic the kernels implement, in Python integers)."""
    rng = random.Random(5)
    for m in (1, 7, 8193):
        b, mods = params(m)
        M = math.prod(mods)
        W = []
        for mt in mods:
            Mt = M // mt
            W.append(Mt * pow(Mt % mt, -1, mt))
        f = [w / M for w in W]
        for _ in range(40):
            x = [rng.randint(-2 ** b, 2 ** b) for _ in range(m)]
            z = [rng.randint(-2 ** b, 2 ** b) for _ in range(m)]
            if rng.random() < 0.3:
                z = x  # diagonal entries
            v = sum(a * c for a, c in zip(x, z))
            ys = []
            for mt in mods:
                c = sum(balanced(a, mt) * balanced(cc, mt) for a, cc in zip(x, z))
                assert abs(c) < 2 ** 31  # int32 accumulation is exact
                ys.append(c % mt)
            qs = 0.0
            for y, ft in zip(ys, f):
                qs = math.fma(y, ft, qs) if hasattr(math, "fma") else qs + y * ft
            Q = round(qs)
            u = (sum(y * w for y, w in zip(ys, W)) - Q * M) % 2 ** 128
            got = u - 2 ** 128 if u >= 2 ** 127 else u
            assert got == v


def test_reconstruction_over_row_chunks():
    """The streamed form at the Boussinesq-type size: 786,689 rows in chunks
    of 32,768, each chunk's residue products summed exactly in int32, the
    chunks added modulo m_t, then the reconstruction recovers the exact sum
    (numpy int64 for the per-row products, Python integers for the rest)."""
    import numpy as np

    m, chunk = 786689, 32768
    b, mods = params(m)
    M = math.prod(mods)
    W = [(M // mt) * pow((M // mt) % mt, -1, mt) for mt in mods]
    f = [w / M for w in W]
    rng = np.random.default_rng(6)
    lim = 2 ** b
    for trial in range(3):
        # integers up to 2^b split into two int64-safe halves for numpy
        x = [int(v) for v in rng.integers(-lim, lim, size=m, dtype=np.int64)]
        z = x if trial == 0 else [int(v) for v in rng.integers(-lim, lim, size=m, dtype=np.int64)]
        v = sum(a * c for a, c in zip(x, z))
        ys = []
        for mt in mods:
            xr = np.array([balanced(a, mt) for a in x], dtype=np.int64)
            zr = xr if z is x else np.array([balanced(a, mt) for a in z], dtype=np.int64)
            y = 0
            for c0 in range(0, m, chunk):
                c = int(np.dot(xr[c0:c0 + chunk], zr[c0:c0 + chunk]))
                assert abs(c) < 2 ** 31  # one chunk's int32 sum is exact
                y = (y + c) % mt
            ys.append(y)
        qs = 0.0
        for y, ft in zip(ys, f):
            qs = math.fma(y, ft, qs) if hasattr(math, "fma") else qs + y * ft
        Q = round(qs)
        u = (sum(y * w for y, w in zip(ys, W)) - Q * M) % 2 ** 128
        got = u - 2 ** 128 if u >= 2 ** 127 else u
        assert got == v
