"""The plain launch's tile schedule: for every workgroup index of a launch
with one workgroup per tile, the tile it runs; together they must cover the
tile triangle (Eq. 11-14) exactly once."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("order") / "liborder_shim.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-Wall",
                    "-I", os.path.join(ROOT, "paper_1704_03767_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "order_shim.cpp"), "-o", out],
                   check=True)
    L = ctypes.CDLL(out)
    ll = ctypes.c_longlong
    L.order_tile.argtypes = [ll, ll, ll, ctypes.POINTER(ll), ctypes.POINTER(ll)]
    L.order_tile.restype = None
    return L


def _tiles(lib, w):
    T = w * (w + 1) // 2
    y, x = ctypes.c_longlong(), ctypes.c_longlong()
    out = np.empty((T, 2), np.int64)
    for b in range(T):
        lib.order_tile(w, T, b, ctypes.byref(y), ctypes.byref(x))
        out[b] = (y.value, x.value)
    return out


@pytest.mark.parametrize("w", list(range(1, 40)) + [63, 64, 65, 100, 127, 160, 257])
def test_schedule_is_a_bijection_onto_the_tile_triangle(lib, w):
    t = _tiles(lib, w)
    assert (t[:, 0] >= 0).all() and (t[:, 0] <= t[:, 1]).all() and (t[:, 1] < w).all()
    flat = t[:, 0] * w + t[:, 1]
    assert np.unique(flat).size == flat.size


def test_each_xcd_walks_bands_in_order(lib):
    # workgroups b, b + 8, b + 16, ... (one XCD) visit consecutive tiles of
    # the band order: inside a band, the tile rows stay within 16 of each other
    w = 300
    t = _tiles(lib, w)
    for x in range(8):
        ys = t[x::8, 0]
        assert (np.diff(ys // 16) >= 0).all()
        xs = t[x::8, 1]
        same_band = np.diff(ys // 16) == 0
        assert (np.diff(xs)[same_band] >= 0).all()
