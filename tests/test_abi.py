"""The C-ABI library loads, exports every symbol its headers declare, and
rejects bad arguments on the host before anything reaches a device."""
import ctypes
import glob
import os
import re

import pytest

from paper_1704_03767_amd import ktau as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(ktau_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert "ktau_allpairs" in names and "ktau_job_to_pair" in names
    lib = ctypes.CDLL(K.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert K.status_string(code) not in ("", "unknown status")
    assert K.status_string(-99) == "unknown status"


def _out():
    return K._PairOut(None, None, None, None, None, None)


def test_host_side_argument_errors():
    L = K.lib()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: rejected first
    ws = ctypes.c_void_p(0x100000)
    assert L.ktau_allpairs(None, 10, 10, _out(), ws, 1 << 20, None) == K.KTAU_EINVAL
    assert L.ktau_allpairs(fake, 1, 10, _out(), ws, 1 << 20, None) == K.KTAU_EINVAL
    assert L.ktau_allpairs(fake, 10, 1, _out(), ws, 1 << 20, None) == K.KTAU_EINVAL
    assert L.ktau_allpairs(fake, 10, K.KTAU_MAX_N + 1, _out(), ws, 1 << 30, None) == K.KTAU_ERANGE
    assert L.ktau_allpairs(fake, 10, 10, _out(), ws, 16, None) == K.KTAU_ENOMEM
    assert L.ktau_allpairs(fake, 10, 10, _out(), ctypes.c_void_p(0x100008), 1 << 20,
                           None) == K.KTAU_EINVAL            # misaligned workspace
    assert L.ktau_allpairs_range(fake, 10, 10, -1, 5, _out(), ws, 1 << 20, None) == K.KTAU_ERANGE
    assert L.ktau_allpairs_range(fake, 10, 10, 5, 46, _out(), ws, 1 << 20, None) == K.KTAU_ERANGE
    assert L.ktau_allpairs_range(fake, 10, 10, 6, 5, _out(), ws, 1 << 20, None) == K.KTAU_ERANGE
    assert L.ktau_allpairs_ex(fake, 300, 300, -1, -1, _out(), ws, 1 << 30, 0, 0,
                              None) == K.KTAU_EINVAL       # wave_k2 holds n <= 128
    assert L.ktau_allpairs_ex(fake, 30, 30, -1, -1, _out(), ws, 1 << 30, 99, 0,
                              None) == K.KTAU_EINVAL
    # the issue-rate probe: kinds 0..3 only, checked before any launch
    assert L.ktau_probe_issue(fake, 1, 1, 4, None) == K.KTAU_EINVAL
    assert L.ktau_probe_issue(fake, 1, 1, -1, None) == K.KTAU_EINVAL
    assert L.ktau_probe_issue(None, 1, 1, 0, None) == K.KTAU_EINVAL
    assert [L.ktau_probe_issue_instrs_per_iter(k) for k in range(-1, 5)] == [-1, 16, 16, 16, 32, -1]
    assert L.ktau_allpairs_ex(fake, 30, 30, -1, -1, _out(), ws, 1 << 30, -1, 65,
                              None) == K.KTAU_EINVAL
    # the naive bit-set scheme takes rows of at most 256 samples
    assert L.ktau_allpairs_ex(fake, 30, 257, -1, -1, _out(), ws, 1 << 30, K.KTAU_SCHEME_NAIVE, 0,
                              None) == K.KTAU_EINVAL
    assert L.ktau_pairs(30, 257, -1, -1, _out(), ws, 1 << 30, K.KTAU_SCHEME_NAIVE, 0,
                        None) == K.KTAU_EINVAL
    assert L.ktau_allpairs_workspace_size(1, 10) == 0
    assert L.ktau_allpairs_workspace_size(10, K.KTAU_MAX_N + 1) == 0
    assert L.ktau_rank(None, 3, 3, None, None, None, None, fake, None, 0, None) == K.KTAU_EINVAL
    assert L.ktau_rank(fake, 3, K.KTAU_MAX_N + 1, None, None, None, None, fake, None, 0,
                       None) == K.KTAU_ERANGE
    # rows longer than 16384 need sort scratch: missing, misaligned, too small
    need = L.ktau_rank_workspace_size(3, 20000)
    assert need >= 3 * 32768 * 8 and L.ktau_rank_workspace_size(3, 16384) == 0
    assert L.ktau_rank(fake, 3, 20000, None, None, None, None, fake, None, need,
                       None) == K.KTAU_EINVAL
    assert L.ktau_rank(fake, 3, 20000, None, None, None, None, fake, ctypes.c_void_p(0x1008), need,
                       None) == K.KTAU_EINVAL
    assert L.ktau_rank(fake, 3, 20000, None, None, None, None, fake, fake, need - 1,
                       None) == K.KTAU_ENOMEM
    # permutation test: host-side argument checks
    need = L.ktau_perm_workspace_size(10, 100, 4)
    assert need > 0 and L.ktau_perm_workspace_size(10, 100, 0) == 0
    assert L.ktau_perm_workspace_size(10, 300, 4) > L.ktau_allpairs_workspace_size(10, 300)
    assert L.ktau_perm_test(fake, 10, 100, None, 4, -1, -1, fake, None, fake, need,
                            None) == K.KTAU_EINVAL
    assert L.ktau_perm_test(fake, 10, 100, fake, 0, -1, -1, fake, None, fake, need,
                            None) == K.KTAU_EINVAL
    assert L.ktau_perm_test(fake, 10, 100, fake, 4, -1, -1, fake, None, fake, need - 1,
                            None) == K.KTAU_ENOMEM
    assert L.ktau_perm_test(fake, 10, 100, fake, 4, 3, 46, fake, None, fake, need,
                            None) == K.KTAU_ERANGE
    assert L.ktau_perm_test(fake, 10, K.KTAU_MAX_N + 1, fake, 4, -1, -1, fake, None, fake,
                            need, None) == K.KTAU_ERANGE
    # the permutation test and the query have network kernels only
    assert L.ktau_perm_workspace_size(10, K.KTAU_MAX_N_NETWORK + 1, 4) == 0
    assert L.ktau_perm_test(fake, 10, K.KTAU_MAX_N_NETWORK + 1, fake, 4, -1, -1, fake, None,
                            fake, need, None) == K.KTAU_ERANGE
    # rows up to KTAU_MAX_N are accepted by the all-pairs calls; their sort
    # scratch covers n rounded up to a power of two
    assert L.ktau_allpairs_workspace_size(10, K.KTAU_MAX_N) > 0
    assert L.ktau_rank_workspace_size(3, 40000) >= 3 * 65536 * 8
    assert L.ktau_pair_to_job(10, 3, 3) == -1
    assert L.ktau_pair_to_job(10, 4, 3) == -1
    assert L.ktau_pair_to_job(10, 3, 10) == -1


def test_scheme_table():
    names = K.ktau_scheme_names()
    assert len(names) == K.lib().ktau_scheme_count()
    caps = [K.ktau_scheme_capacity(i) for i in range(len(names))]
    assert max(caps) >= K.KTAU_MAX_N
    for n in (2, 64, 128, 129, 512, 1024, 1025, 4096, 4097, 8192, 8193, 16384, 32769, 65536):
        s = K.ktau_default_scheme(n)
        assert caps[s] >= n
    assert names[-2:] == ["merge_k32", "merge_k64"]
    assert caps[-2:] == [32768, 65536]
    assert K.ktau_scheme_capacity(-1) == -1


def test_workspace_holds_the_bit_sets():
    # rows of <= 256 samples: two sets of ceil(n/32) words (rounded to 1, 2, 4
    # or 8) per sample behind the rank layout
    for n, words in ((32, 1), (33, 2), (64, 2), (100, 4), (128, 4), (129, 8), (256, 8)):
        m = 50
        assert K.ktau_allpairs_workspace_size(m, n) >= 2 * m * n * words * 4 + 3 * m * 128 * 2
    big = K.ktau_allpairs_workspace_size(50, 257)
    assert big < K.ktau_allpairs_workspace_size(50, 256)
    assert K.ktau_plain_default_scheme(1024) == K.ktau_default_scheme(1024)
    # the plain calls take the naive bit-set count up to n = 128 (where it
    # measured faster), the network beyond
    for n in (2, 32, 64, 100, 128):
        assert K.ktau_plain_default_scheme(n) == K.KTAU_SCHEME_NAIVE
    for n in (129, 256, 4096):
        assert K.ktau_plain_default_scheme(n) == K.ktau_default_scheme(n)
    assert K.scheme_id(K.NAIVE_SCHEME_NAME) == K.KTAU_SCHEME_NAIVE


def test_plain_default_tile_edge():
    # 16 x 16 tiles from 8192 rows on (networks up to 4096 samples), 8 x 8
    # below; the bit-set count keeps 16; longer rows take smaller tiles
    assert K.ktau_plain_default_q(16384, 1024) == 16
    assert K.ktau_plain_default_q(17941, 353) == 16
    assert K.ktau_plain_default_q(8191, 1024) == 8
    assert K.ktau_plain_default_q(4096, 512) == 8
    assert K.ktau_plain_default_q(64, 128) == 16
    assert K.ktau_plain_default_q(16384, 8192) == 4
    assert K.ktau_plain_default_q(353, 17941) == 2


def test_workspace_size_grows_with_shape():
    a = K.ktau_allpairs_workspace_size(64, 128)
    b = K.ktau_allpairs_workspace_size(16384, 1024)
    assert 0 < a < b
    assert b >= 3 * 16384 * 1024 * 2
