"""The allocation-free all-pairs entry point (ktau_allpairs_noalloc) through
the C ABI: results equal ktau_allpairs' bit for bit on two calls in a row, the
second with a smaller input; shapes beyond its static scratch are refused
before any launch; a NaN input is reported through its status word."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu
KEYS = ("nc", "nd", "n3", "tau_b", "tau_a", "n1")


def _lib():
    L = K.lib()
    f = L.ktau_allpairs_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, K._PairOut, ctypes.c_void_p,
                  ctypes.c_void_p]
    f.restype = ctypes.c_int
    return L


def _noalloc(X: torch.Tensor):
    m, n = X.shape
    out = K.alloc_outputs(m * (m - 1) // 2, m, X.device, tau_a=True)
    status = torch.full((1,), -99, dtype=torch.int32, device=X.device)
    rc = _lib().ktau_allpairs_noalloc(ctypes.c_void_p(X.data_ptr()), m, n, K._pair_out(out),
                                      ctypes.c_void_p(status.data_ptr()), K._stream())
    torch.cuda.synchronize()
    return rc, out, int(status.item())


def _same(a, b):
    for k in KEYS:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True), k


def test_noalloc_equals_plain_on_two_calls_the_second_smaller():
    shapes = [(300, 700, 81), (37, 129, 82)]
    for m, n, seed in shapes:
        X = torch.from_numpy(synth.lognormal_blocks(m, n, seed)).cuda()
        rc, got, st = _noalloc(X)
        assert rc == K.KTAU_OK and st == K.KTAU_OK
        want = K.ktau_allpairs(X, tau_a=True)
        _same(got, want)


def test_noalloc_long_rows_and_ties():
    # rows beyond one wave's network (merge scheme) and heavily tied rows
    rng = np.random.default_rng(83)
    X = np.round(rng.standard_normal((12, 9000)), 1).astype(np.float32)
    X[3] = 1.0
    X[4] = rng.integers(0, 2, 9000).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    rc, got, st = _noalloc(Xd)
    assert rc == K.KTAU_OK and st == K.KTAU_OK
    _same(got, K.ktau_allpairs(Xd, tau_a=True))


def test_noalloc_refuses_shapes_beyond_its_scratch_and_reports_nan():
    L = _lib()
    big = K.ktau_allpairs_workspace_size(16384, 1024)
    assert big > 64 << 20
    fake = ctypes.c_void_p(0x1000)    # never dereferenced: refused before any launch
    assert L.ktau_allpairs_noalloc(fake, 16384, 1024, K._PairOut(None, None, None, None, None,
                                                                 None), None,
                                   None) == K.KTAU_ENOMEM
    X = synth.config_matrix(1).copy()
    X[5, 7] = np.nan
    rc, _, st = _noalloc(torch.from_numpy(X).cuda())
    assert rc == K.KTAU_OK and st == K.KTAU_ENAN
    # the status was taken and cleared: the next call is clean
    rc, got, st = _noalloc(torch.from_numpy(synth.config_matrix(1)).cuda())
    assert rc == K.KTAU_OK and st == K.KTAU_OK
    _same(got, K.ktau_allpairs(torch.from_numpy(synth.config_matrix(1)).cuda(), tau_a=True))
