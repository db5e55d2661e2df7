"""Job-id bijection of the library (Sec. 4.1 Eq. 4-10, strict triangle; tiles
Sec. 4.2 Eq. 11-14) against the oracle's row-major enumeration.  Host code of
libktau.so only -- no GPU needed."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1704_03767_amd import ktau as K


def _lib():
    return K.lib()


def test_exhaustive_small_m():
    L = _lib()
    y, x = ctypes.c_int64(), ctypes.c_int64()
    for m in list(range(2, 70)) + [127, 128, 129, 255, 256, 257]:
        ys, xs = oracle.enumerate_pairs(m)
        for J in range(len(ys)):
            assert L.ktau_pair_to_job(m, int(ys[J]), int(xs[J])) == J
            assert L.ktau_job_to_pair(m, J, ctypes.byref(y), ctypes.byref(x)) == 0
            assert (y.value, x.value) == (ys[J], xs[J])
        assert L.ktau_job_to_pair(m, len(ys), ctypes.byref(y), ctypes.byref(x)) == K.KTAU_ERANGE
        assert L.ktau_job_to_pair(m, -1, ctypes.byref(y), ctypes.byref(x)) == K.KTAU_ERANGE


@pytest.mark.parametrize("m", [511, 1024, 2048])
def test_exhaustive_large_m(m):
    # every job of an m up to 2048 (about 2.1M jobs), checked in bulk
    L = _lib()
    ys, xs = oracle.enumerate_pairs(m)
    y, x = ctypes.c_int64(), ctypes.c_int64()
    bad = 0
    step = 1 if m <= 1024 else 3
    for J in range(0, len(ys), step):
        L.ktau_job_to_pair(m, J, ctypes.byref(y), ctypes.byref(x))
        bad += (y.value != ys[J]) or (x.value != xs[J])
    assert bad == 0


def test_row_boundaries_up_to_2_pow_20():
    L = _lib()
    y, x = ctypes.c_int64(), ctypes.c_int64()
    rng = np.random.default_rng(0)
    for m in [2 ** k + d for k in range(11, 21) for d in (-1, 0, 1)] + [16384, 17941, 20000]:
        rows = set(int(r) for r in rng.integers(0, m - 1, 40)) | {0, 1, m // 2, m - 3, m - 2}
        for r in rows:
            if r < 0 or r > m - 2:
                continue
            start = r * (m - 1) - r * (r - 1) // 2          # row-major count before row r
            for J, want in ((start, (r, r + 1)), (start + (m - 2 - r), (r, m - 1))):
                assert L.ktau_job_to_pair(m, J, ctypes.byref(y), ctypes.byref(x)) == 0
                assert (y.value, x.value) == want, (m, r, J)
                assert L.ktau_pair_to_job(m, *want) == J
            if r > 0:
                assert L.ktau_job_to_pair(m, start - 1, ctypes.byref(y), ctypes.byref(x)) == 0
                assert (y.value, x.value) == (r - 1, m - 1)
    P = (2 ** 20) * (2 ** 20 - 1) // 2
    assert L.ktau_job_to_pair(2 ** 20, P - 1, ctypes.byref(y), ctypes.byref(x)) == 0
    assert (y.value, x.value) == (2 ** 20 - 2, 2 ** 20 - 1)


def test_tiles_inclusive_triangle():
    L = _lib()
    y, x = ctypes.c_int64(), ctypes.c_int64()
    for w in list(range(1, 80)) + [1024, 2048]:
        t = 0
        rows = range(w) if w < 100 else [0, 1, w // 2, w - 2, w - 1]
        for yq in range(w):
            if yq not in rows:
                t += w - yq
                continue
            for xq in range(yq, w):
                assert L.ktau_tile_to_coord(w, t, ctypes.byref(y), ctypes.byref(x)) == 0
                assert (y.value, x.value) == (yq, xq)
                t += 1
        assert t == w * (w + 1) // 2
        assert L.ktau_tile_to_coord(w, t, ctypes.byref(y), ctypes.byref(x)) == K.KTAU_ERANGE


def test_tiles_cover_every_strict_pair_once():
    for m, q in [(2, 8), (9, 8), (64, 8), (65, 4), (100, 16), (37, 1)]:
        w = -(-m // q)
        seen = []
        for t in range(w * (w + 1) // 2):
            yq, xq = K.ktau_tile_to_coord(w, t)
            for a in range(q):
                for b in range(q):
                    yy, xx = yq * q + a, xq * q + b
                    if yy < xx < m:
                        seen.append(K.ktau_pair_to_job(m, yy, xx))
        assert sorted(seen) == list(range(m * (m - 1) // 2))
