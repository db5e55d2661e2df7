"""The query server's scheduling core on the CPU, with a fake executor whose
launches finish only when the test says so: arrival order, merging of
consecutive same-k requests, admission by memory, slot reuse, isolation of a
forced failure, cancellation, and the first-fit pool."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
QUEUED, RUNNING, DONE = 1, 2, 0


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("sched") / "libsched_shim.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-Wall",
                    "-I", os.path.join(ROOT, "paper_1704_03767_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "sched_shim.cpp"), "-o", out],
                   check=True)
    L = ctypes.CDLL(out)
    ll, i = ctypes.c_longlong, ctypes.c_int
    p = ctypes.c_void_p
    for name, args, res in [
        ("st_create", [i, ll, ll, ll], p), ("st_submit", [p, ll, ll, i], ll),
        ("st_step", [p], i), ("st_finish_slot", [p, i], None), ("st_state", [p, ll], i),
        ("st_status", [p, ll], i), ("st_batch_requests", [p, ll], ll),
        ("st_batch_queries", [p, ll], ll), ("st_result0", [p, ll], ll),
        ("st_pool_used", [p], ll), ("st_running", [p], ll), ("st_queued", [p], ll),
        ("st_cancel", [p, ll], i), ("st_peak_running", [p], ll), ("st_destroy", [p], None),
        ("st_pool_fuzz", [ll, i, ctypes.c_uint], i), ("st_fail_start", [p, ll], None),
        ("st_overlaps", [p], i), ("st_abandoned", [p], i), ("st_inflight", [p], i),
        ("st_pause", [p, i], None), ("st_launch_k", [p, ll], ll),
    ]:
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


def test_merging_and_fifo(lib):
    w = lib.st_create(2, 10, 1 << 30, 1000)
    t = [lib.st_submit(w, nq, 100, 0) for nq in (3, 4, 2, 5, 1)]
    lib.st_step(w)
    # slot 0: 3+4+2 = 9 rows (the 5 would exceed 10); slot 1: 5+1
    assert [lib.st_state(w, x) for x in t] == [RUNNING] * 5
    assert [lib.st_batch_requests(w, x) for x in t] == [3, 3, 3, 2, 2]
    assert [lib.st_batch_queries(w, x) for x in t] == [9, 9, 9, 6, 6]
    lib.st_finish_slot(w, 1)
    assert lib.st_step(w) == 2
    assert lib.st_state(w, t[3]) == DONE and lib.st_state(w, t[0]) == RUNNING
    assert lib.st_result0(w, t[4]) == t[4]
    lib.st_finish_slot(w, 0)
    assert lib.st_step(w) == 3
    assert lib.st_pool_used(w) == 0 and lib.st_running(w) == 0
    lib.st_destroy(w)


def test_different_k_merge_at_the_largest_k(lib):
    w = lib.st_create(4, 64, 1 << 30, 1000)
    t = [lib.st_submit(w, 2, k, 0) for k in (10, 10, 20, 10)]
    lib.st_step(w)
    assert [lib.st_batch_requests(w, x) for x in t] == [4, 4, 4, 4]
    lib.st_finish_slot(w, 0)
    assert lib.st_step(w) == 4
    # the launch ran k = 20; every request still gets its own k per row
    assert [lib.st_launch_k(w, x) for x in t] == [20, 20, 20, 20]
    lib.st_destroy(w)


def test_admission_by_memory(lib):
    # each launch of 4 rows needs 4000 B; 10000 B budget fits two at a time
    w = lib.st_create(8, 4, 10_000, 1000)
    t = [lib.st_submit(w, 4, 5, 0) for _ in range(6)]
    lib.st_step(w)
    assert lib.st_running(w) == 2 and lib.st_queued(w) == 4
    assert lib.st_pool_used(w) <= 10_000
    for round_ in range(3):
        for s in range(8):
            lib.st_finish_slot(w, s)
        lib.st_step(w)
        assert lib.st_pool_used(w) <= 10_000
    while lib.st_running(w):
        for s in range(8):
            lib.st_finish_slot(w, s)
        lib.st_step(w)
    assert all(lib.st_state(w, x) == DONE and lib.st_status(w, x) == 0 for x in t)
    assert lib.st_peak_running(w) == 2
    # a request that can never fit is refused
    assert lib.st_submit(w, 11, 5, 0) == -1
    lib.st_destroy(w)


def test_head_waits_for_memory_and_keeps_order(lib):
    w = lib.st_create(4, 64, 10_000, 1000)
    a = lib.st_submit(w, 8, 5, 0)           # 8000 B
    lib.st_step(w)
    b = lib.st_submit(w, 5, 5, 0)           # 5000 B does not fit beside a
    c = lib.st_submit(w, 1, 6, 0)           # would fit, but must not overtake b
    lib.st_step(w)
    assert lib.st_state(w, b) == QUEUED and lib.st_state(w, c) == QUEUED
    lib.st_finish_slot(w, 0)
    lib.st_step(w)
    assert lib.st_state(w, a) == DONE
    assert lib.st_state(w, b) == RUNNING and lib.st_state(w, c) == RUNNING
    lib.st_destroy(w)


def test_forced_failure_runs_alone(lib):
    w = lib.st_create(1, 64, 1 << 30, 1000)
    x = lib.st_submit(w, 1, 5, 0)
    lib.st_step(w)                          # x occupies the only slot
    a = lib.st_submit(w, 2, 5, 0)
    f = lib.st_submit(w, 2, 5, 1)
    b = lib.st_submit(w, 2, 5, 0)
    lib.st_finish_slot(w, 0)
    lib.st_step(w)                          # x done; a launched alone (f never merges)
    assert lib.st_batch_requests(w, a) == 1
    lib.st_finish_slot(w, 0)
    lib.st_step(w)                          # a done; f launched alone
    lib.st_step(w)                          # f collected as failed; b launched
    assert lib.st_status(w, f) == -7 and lib.st_state(w, f) == DONE
    lib.st_finish_slot(w, 0)
    lib.st_step(w)
    assert lib.st_status(w, a) == 0 and lib.st_status(w, b) == 0
    assert lib.st_result0(w, b) == b
    lib.st_destroy(w)


def test_cancel_only_while_queued(lib):
    w = lib.st_create(1, 1, 1 << 30, 1000)     # one row per launch: b waits
    a = lib.st_submit(w, 1, 5, 0)
    b = lib.st_submit(w, 1, 7, 0)
    lib.st_step(w)
    assert lib.st_cancel(w, a) == 0         # running
    assert lib.st_cancel(w, b) == 1         # queued
    assert lib.st_queued(w) == 0
    lib.st_destroy(w)


def test_pool_first_fit(lib):
    for seed in range(5):
        assert lib.st_pool_fuzz(1 << 20, 2000, seed) == 1


def test_failed_start_is_drained_before_its_region_is_reused(lib):
    # a launch whose start enqueues work and then fails must be drained by the
    # executor before its pool region is handed to another launch
    w = lib.st_create(2, 64, 4_096, 1000)
    a = lib.st_submit(w, 4, 5, 0)           # 4000 B: the whole pool (4096)
    lib.st_fail_start(w, a)
    b = lib.st_submit(w, 4, 7, 0)           # needs the same region
    lib.st_step(w)                          # a starts, fails, is drained
    assert lib.st_abandoned(w) == 1 and lib.st_inflight(w) == 0
    assert lib.st_state(w, b) == QUEUED
    lib.st_step(w)                          # a collected as failed; b admitted
    assert lib.st_status(w, a) == -7 and lib.st_state(w, a) == DONE
    assert lib.st_state(w, b) == RUNNING
    assert lib.st_overlaps(w) == 0
    lib.st_finish_slot(w, 0)
    lib.st_finish_slot(w, 1)
    lib.st_step(w)
    assert lib.st_status(w, b) == 0 and lib.st_pool_used(w) == 0
    lib.st_destroy(w)


def test_pause_holds_admission_and_resume_merges(lib):
    w = lib.st_create(2, 64, 1 << 30, 1000)
    lib.st_pause(w, 1)
    t = [lib.st_submit(w, nq, 100, 0) for nq in (2, 3, 4)]
    lib.st_step(w)
    assert [lib.st_state(w, x) for x in t] == [QUEUED] * 3 and lib.st_running(w) == 0
    lib.st_pause(w, 0)
    lib.st_step(w)
    assert [lib.st_batch_requests(w, x) for x in t] == [3, 3, 3]
    # a running launch still completes while admission is paused
    lib.st_pause(w, 1)
    u = lib.st_submit(w, 1, 100, 0)
    lib.st_finish_slot(w, 0)
    assert lib.st_step(w) == 3 and lib.st_state(w, u) == QUEUED
    lib.st_pause(w, 0)
    lib.st_step(w)
    assert lib.st_state(w, u) == RUNNING
    lib.st_destroy(w)
