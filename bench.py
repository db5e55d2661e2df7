#!/usr/bin/env python
"""Throughput of exact all-pairs Kendall's tau on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the hot path over the gene-expression-scale workload
(m = 16384 variables x n = 1024 samples, log-normal rows in correlated blocks
of 64 with 2% exact zeros, seed 3): the rank pre-pass of every row, then the
pair kernel over all 134,209,536 strict pairs writing int64 n_c, n_d, n3 and
FP64 tau_B.  Inputs are resident in HBM before the timed region; outputs stay
in HBM.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = ("tau pairs/sec at m=16384,n=1024 (batched vs plain, exact); "
          "p50/p99 query latency")

# MI355X published figures used for the roofline denominators.
CUS = 256
CLOCK_HZ = 2.4e9
# Integer VALU: 4 SIMDs per CU, each retiring one 64-lane wave instruction
# every 4 cycles = 64 int32 lane-ops per CU per cycle.
INT_VALU_OPS = CUS * 64 * CLOCK_HZ           # 3.93e13 lane-ops/s
# LDS reference width: 128 bytes per cycle per CU (the CDNA3 figure; the
# probe measures what gfx950 reaches).
LDS_BYTES_PER_S = CUS * 128 * CLOCK_HZ       # 7.86e13 B/s
# The paper's VSE kernel on one Xeon Phi 5110P for its 17,941 x 353 dataset
# (Table 4: 296 s), as strict pairs per second: context, not a target.
PAPER_PHI_DS3526 = 17941 * 17940 / 2 / 296.0


def merge_steps(n: int) -> int:
    """Algorithmic compare-and-move steps of one pair's merge-sort count."""
    return n * math.ceil(math.log2(n))


# The sources the all-pairs kernel is built from (the public header adds only
# declarations and status codes): a committed counter summary holds for the
# kernel only while these are unchanged.
PAIR_KERNEL_SOURCES = ("paper_1704_03767_amd/csrc/ktau_pair.hip",
                       "paper_1704_03767_amd/csrc/ktau_pairdev.h",
                       "paper_1704_03767_amd/csrc/ktau_bitonic.h",
                       "paper_1704_03767_amd/csrc/ktau_internal.h",
                       "paper_1704_03767_amd/csrc/ktau_order.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in PAIR_KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_tag: str, src_hash: str):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_hash") != src_hash:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(X, seconds: float, gpu: dict | None = None, seed: int = 99) -> dict:
    """The oracle (sorting kernel, all host threads) on a seeded sample of
    pairs.  With gpu (the timed run's device outputs: nc, nd, n3, tau_b by job
    id and n1 per row) the first batch of sampled pairs is also compared with
    them: the parity record of the run that was timed."""
    import numpy as np

    import oracle

    m, n = X.shape
    threads = oracle.max_threads()
    rng = np.random.default_rng(seed)
    parity = None

    def run(count, check=False):
        nonlocal parity
        ys = rng.integers(0, m - 1, count)
        xs = ys + 1 + (rng.integers(0, 1 << 62, count) % (m - 1 - ys))
        t0 = time.perf_counter()
        want = oracle.pairs(X, ys, xs, "gse", threads)
        dt = time.perf_counter() - t0
        if check and gpu is not None:
            import torch

            J = ys * (2 * (m - 1) - ys + 1) // 2 + (xs - 1 - ys)   # strict job ids
            Jd = torch.from_numpy(J).to(gpu["nc"].device)
            same = all(np.array_equal(gpu[k][Jd].cpu().numpy(), want[k])
                       for k in ("nc", "nd", "n3"))
            n1 = gpu["n1"].cpu().numpy()
            same = same and np.array_equal(n1[ys], want["n1"]) and np.array_equal(n1[xs],
                                                                                  want["n2"])
            tg, tw = gpu["tau_b"][Jd].cpu().numpy(), want["tau_b"]
            nan_same = bool(np.array_equal(np.isnan(tg), np.isnan(tw)))
            ok = ~np.isnan(tw)
            parity = {"pairs": int(count), "counts_equal": bool(same),
                      "tau_nan_equal": nan_same,
                      "max_abs_dtau": float(np.abs(tg[ok] - tw[ok]).max()) if ok.any() else 0.0,
                      "what": "n_c, n_d, n3, n1, n2 and tau_B of the timed (batched) run at "
                              "the oracle's first batch of seeded pairs"}
        return dt

    # batches of seeded pairs, each sized from the rate so far, until about
    # `seconds` of oracle time have been spent
    count, dt, batch = 0, 0.0, max(threads * 64, 1024)
    first = True
    while dt < seconds:
        dt += run(batch, check=first)
        first = False
        count += batch
        left = seconds - dt
        batch = int(min(20_000_000, max(threads * 64, 1.1 * left * count / max(dt, 1e-6))))
    res = {"value": count / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
           "sample": f"{count} seeded random strict pairs of the same matrix, "
                     f"sorting-kernel routine, {dt:.1f} s on {threads} threads",
           "cpu": cpu_model(), "nproc": os.cpu_count()}
    if parity is not None:
        res["parity"] = parity
    return res


def outputs_equal(a: dict, b: dict) -> bool:
    """Bitwise equality of two device output sets (NaN tau_B at the same
    slots)."""
    import torch

    for k in ("nc", "nd", "n3", "n1"):
        if k in a and k in b and not torch.equal(a[k], b[k]):
            return False
    ta, tb = a["tau_b"], b["tau_b"]
    if not torch.equal(ta.isnan(), tb.isnan()):
        return False
    ok = ~ta.isnan()
    return bool(torch.equal(ta[ok], tb[ok]))


def uneven_batch(K, synth, torch, stream, reps: int) -> dict:
    """256 matrices, m ~ U[32, 2048], n ~ U[64, 4096], N(0,1) with 20% of the
    entries on a 0.25 grid (seed 4): 256 plain calls vs one batched plan."""
    import numpy as np

    mats = synth.batch(256, 4)
    dev = [torch.from_numpy(X).cuda() for X in mats]
    del mats
    outs = [K.alloc_outputs(X.shape[0] * (X.shape[0] - 1) // 2, X.shape[0], X.device)
            for X in dev]
    outs_b = [K.alloc_outputs(X.shape[0] * (X.shape[0] - 1) // 2, X.shape[0], X.device)
              for X in dev]
    pairs = sum(X.shape[0] * (X.shape[0] - 1) // 2 for X in dev)
    steps = sum(X.shape[0] * (X.shape[0] - 1) // 2 * merge_steps(X.shape[1]) for X in dev)
    ws = torch.empty(max(K.ktau_allpairs_workspace_size(*X.shape) for X in dev),
                     dtype=torch.uint8, device="cuda")

    def plain():
        for X, o in zip(dev, outs):
            K.ktau_prepare(X, ws, o["n1"], stream=stream)
            K.ktau_pairs(X.shape[0], X.shape[1], o, ws, stream=stream)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_plain = timed(plain)
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError("uneven batch: plain calls failed")
    plan = K.KtauBatch(dev, outs=outs_b, stream=stream)
    ms_batch = timed(lambda: plan.run(stream))
    if plan.status(stream) != K.KTAU_OK:
        raise RuntimeError("uneven batch: batched run failed")
    classes = sorted({plan.plan(i) for i in range(len(dev))})
    plan.close()
    same = all(outputs_equal(a, b) for a, b in zip(outs, outs_b))
    return {"workload": "256 matrices m~U[32,2048] n~U[64,4096], 20% of entries on a 0.25 grid, "
                        "seed 4",
            "pairs": pairs, "merge_steps": steps,
            "plain_ms": ms_plain, "plain_pairs_per_s": pairs / (ms_plain * 1e-3),
            "batched_ms": ms_batch, "batched_pairs_per_s": pairs / (ms_batch * 1e-3),
            "speedup": ms_plain / ms_batch,
            "batched_equals_plain": same,
            "plans": [f"{s}/q{q}" for s, q in classes]}


def scheme_label(K, scheme: int) -> str:
    return K.NAIVE_SCHEME_NAME if scheme == K.KTAU_SCHEME_NAIVE else K.ktau_scheme_names()[scheme]


def plain_timing(K, torch, stream, X, reps: int) -> dict:
    """Mean time of the plain path (pre-pass + pair kernel) on matrix X."""
    Xd = torch.from_numpy(X).cuda()
    m, n = X.shape
    P = m * (m - 1) // 2
    out = K.alloc_outputs(P, m, Xd.device)
    ws = K.alloc_workspace(m, n, Xd.device)

    def step():
        K.ktau_prepare(Xd, ws, out["n1"], stream=stream)
        K.ktau_pairs(m, n, out, ws, stream=stream)

    step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError(f"plain call on {m} x {n} failed")
    ms = e0.elapsed_time(e1) / reps
    return {"m": m, "n": n, "pairs": P, "ms": ms, "pairs_per_s": P / (ms * 1e-3),
            "scheme": scheme_label(K, K.ktau_plain_default_scheme(n)),
            "merge_steps_per_s": P * merge_steps(n) / (ms * 1e-3)}


def split_timing(K, torch, stream, X, reps: int, scheme=None) -> dict:
    """The plain path on matrix X with the pre-pass and the pair kernel timed
    apart (HIP events on the launching stream); outputs in HBM."""
    import numpy as np

    Xd = torch.from_numpy(X).cuda()
    m, n = X.shape
    P = m * (m - 1) // 2
    out = K.alloc_outputs(P, m, Xd.device)
    ws = K.alloc_workspace(m, n, Xd.device)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps + 1)]
    for e in ev:
        e[0].record(stream)
        K.ktau_prepare(Xd, ws, out["n1"], stream=stream)
        e[1].record(stream)
        K.ktau_pairs(m, n, out, ws, scheme=scheme, stream=stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError(f"plain call on {m} x {n} failed")
    prep = [e[0].elapsed_time(e[1]) for e in ev[1:]]
    pair = [e[1].elapsed_time(e[2]) for e in ev[1:]]
    ms = float(np.mean(prep)) + float(np.mean(pair))
    pair_ms = float(np.mean(pair))
    steps = P * merge_steps(n)
    used = K.ktau_plain_default_scheme(n) if scheme is None else K.scheme_id(scheme)
    return {"m": m, "n": n, "pairs": P, "ms": ms, "pairs_per_s": P / (ms * 1e-3),
            "prepass_ms": float(np.mean(prep)), "pair_kernel_ms": pair_ms,
            "pair_kernel_ms_min": float(np.min(pair)),
            "scheme": scheme_label(K, used),
            "merge_steps_per_s": steps / (pair_ms * 1e-3),
            "frac": steps / (pair_ms * 1e-3) / INT_VALU_OPS, "out": out}


def medium(K, synth, torch, stream, reps: int) -> dict:
    """The medium workload: m = 4096 x n = 512 from a latent-factor model (8
    factors, noise sd 0.5), 10% of the rows quantised to 16 levels (seed 2):
    the plain path (pre-pass and pair kernel apart) and the batched form,
    whose results must equal the plain call's bit for bit."""
    X = synth.config_matrix(2)
    r = split_timing(K, torch, stream, X, reps)
    plain_out = r.pop("out")
    Xd = torch.from_numpy(X).cuda()
    m = X.shape[0]
    out_b = K.alloc_outputs(m * (m - 1) // 2, m, Xd.device)
    plan = K.KtauBatch([Xd], outs=[out_b], stream=stream)
    plan.run(stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.run(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    if plan.status(stream) != K.KTAU_OK:
        raise RuntimeError("medium: batched run failed")
    ms_b = e0.elapsed_time(e1) / reps
    r["batched"] = {"ms": ms_b, "pairs_per_s": r["pairs"] / (ms_b * 1e-3),
                    "scheme": plan.plan(0)[0], "q": plan.plan(0)[1],
                    "equals_plain": outputs_equal(out_b, plain_out)}
    plan.close()
    r["workload"] = ("medium m=4096 n=512 latent factors (8, noise sd 0.5), 10% of rows "
                     "quantised to 16 levels, seed 2")
    r["ops_per_pair"] = merge_steps(X.shape[1])
    r["input_sha256"] = synth.sha256(X)[:16]
    return r


def large_n(K, synth, torch, stream, reps: int) -> dict:
    """Rows beyond one wave's network: the merge scheme (chunk networks and a
    merge path over them) on log-normal rows of 32768 and 65536 samples (the
    second with plain 16-bit ranks counted in two halves)."""
    rows = []
    for m, n in ((200, 32768), (96, 65536)):
        r = split_timing(K, torch, stream, synth.lognormal_blocks(m, n, 3), reps)
        r.pop("out")
        r["workload"] = (f"m={m} n={n} log-normal, blocks of 64 rows at rho=0.6, 2% exact zeros, "
                         "seed 3")
        rows.append(r)
    return {"rows": rows}


def other_shapes(K, synth, torch, stream, reps: int) -> dict:
    """The paper's two orientations of its gene-expression data: genes as
    variables (m = 17,941, n = 353, as its timed datasets; its one-Phi VSE
    rate for that shape, derived from Table 4, is context) and samples as
    variables (m = 353, n = 17,941: the merge scheme, pre-pass and pair kernel
    timed apart)."""
    genes = plain_timing(K, torch, stream, synth.lognormal_blocks(17941, 353, 7), reps)
    genes["workload"] = ("gene-vs-gene m=17941 n=353 log-normal, blocks of 64 rows at rho=0.6, "
                         "2% exact zeros, seed 7")
    genes["paper_phi_vse_pairs_per_s"] = PAPER_PHI_DS3526
    samples = split_timing(K, torch, stream, synth.samples_matrix(353, 17941, 6), reps)
    samples.pop("out")
    samples["workload"] = ("sample-vs-sample m=353 n=17941: per-gene level + 4 group offsets + "
                           "noise, exp, 2% exact zeros, seed 6")
    return {"gene_vs_gene": genes, "sample_vs_sample": samples}


def small_n(K, synth, torch, stream, reps: int) -> dict:
    """Short rows: the naive count (every sample pair compared, Sec. 3.1) from
    per-row bit sets against the default network scheme, pair kernel alone on
    4096 log-normal rows (blocks of 64 at rho 0.6, 2% exact zeros) per n; and
    the 64 x 128 rounded-normal case end to end (pre-pass + pairs), which is
    launch-bound."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = []
    for n in (32, 64, 128, 256):
        X = synth.lognormal_blocks(4096, n, 500 + n)
        m = X.shape[0]
        P = m * (m - 1) // 2
        Xd = torch.from_numpy(X).cuda()
        ws = K.alloc_workspace(m, n, Xd.device)
        out = K.alloc_outputs(P, m, Xd.device)
        K.ktau_prepare(Xd, ws, out["n1"], stream=stream)
        net = K.ktau_default_scheme(n)
        row = {"n": n, "m": m, "pairs": P, "network_scheme": K.ktau_scheme_names()[net]}
        for name, scheme in (("naive_bits", K.NAIVE_SCHEME_NAME), ("network", net)):
            ms = timed(lambda: K.ktau_pairs(m, n, out, ws, scheme=scheme, stream=stream))
            row[f"{name}_ms"] = ms
            row[f"{name}_pairs_per_s"] = P / (ms * 1e-3)
        if K.ktau_status(ws) != K.KTAU_OK:
            raise RuntimeError(f"short-row timing on {m} x {n} failed")
        row["naive_speedup"] = row["network_ms"] / row["naive_bits_ms"]
        rows.append(row)
    X = synth.config_matrix(1)
    m, n = X.shape
    P = m * (m - 1) // 2
    Xd = torch.from_numpy(X).cuda()
    ws = K.alloc_workspace(m, n, Xd.device)
    out = K.alloc_outputs(P, m, Xd.device)
    c1 = {"m": m, "n": n, "pairs": P}
    for name, scheme in (("naive_bits", K.NAIVE_SCHEME_NAME),
                         ("network", K.ktau_default_scheme(n))):
        c1[f"{name}_us"] = 1e3 * timed(
            lambda: K.ktau_allpairs_ex(Xd, -1, -1, out, ws, scheme, 0, stream))
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError("64 x 128 timing failed")
    return {"workload": "m=4096 log-normal blocks (seed 500+n), pair kernel alone; "
                        "64x128 rounded normals (seed 1) end to end",
            "rows": rows, "c1_64x128": c1}


def perm_test(K, synth, torch, stream, reps: int) -> dict:
    """Permutation-test P-values (Sec. 1): m = 512 log-normal rows (blocks of
    64 at rho = 0.6, 2% exact zeros, seed 11) of n = 1024 samples, B = 200
    permutations (seed 12) of the second row of every pair: 201 tau counts
    per pair."""
    X = synth.lognormal_blocks(512, 1024, 11)
    perms = synth.permutations(200, 1024, 12)
    m, n = X.shape
    B = perms.shape[0]
    P = m * (m - 1) // 2
    Xd = torch.from_numpy(X).cuda()
    Pd = torch.from_numpy(perms.astype("int16")).cuda()
    size = K.lib().ktau_perm_workspace_size(m, n, B)
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    count = torch.empty(P, dtype=torch.int64, device="cuda")
    p = torch.empty(P, dtype=torch.float64, device="cuda")

    def run():
        rc = K.lib().ktau_perm_test(K._ptr(Xd), m, n, K._ptr(Pd), B, -1, -1, K._ptr(count),
                                    K._ptr(p), K._ptr(ws), size, K._stream(stream))
        if rc != K.KTAU_OK:
            raise RuntimeError(f"ktau_perm_test: {K.status_string(rc)}")

    run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError("permutation test failed on the device")
    ms = e0.elapsed_time(e1) / reps
    taus = P * (B + 1)
    return {"workload": "m=512 n=1024 log-normal (blocks of 64, rho=0.6, 2% zeros, seed 11), "
                        "B=200 permutations (seed 12)",
            "pairs": P, "permutations": B, "ms": ms, "tau_per_s": taus / (ms * 1e-3),
            "scheme": K.ktau_scheme_names()[K.ktau_default_scheme(n)],
            "median_p": float(p.median().item())}


def serving(K, synth, torch, stream, seconds: float) -> dict:
    """Query-vs-database search over a resident 20000 x 800 log-normal
    database (seed 5): requests of 1-64 query rows, top-100 by |tau_B|.
    Closed-loop saturation of the server, one plain ktau_query launch per
    request for comparison, then Poisson arrivals at 0.5x and 0.8x saturation
    with per-request latency = completion - submission (queueing included)."""
    import threading

    import numpy as np

    from paper_1704_03767_amd import serve as S

    k = 100
    db = synth.database(20000, 800, 5)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda(), stream=stream)
    m = db.X.shape[0]
    rng = np.random.default_rng(55)
    pool_sizes = rng.integers(1, 65, 4096)
    Qpool = synth.queries(db, int(pool_sizes.sum()), 56)
    offs = np.concatenate([[0], np.cumsum(pool_sizes)])
    req = [Qpool[offs[i]:offs[i + 1]] for i in range(len(pool_sizes))]

    # plain: one stream-ordered launch per request, waited for
    n_plain = 64
    ws = torch.empty(S.ktau_query_workspace_size(kdb, 64, k), dtype=torch.uint8, device="cuda")
    qdev = [torch.from_numpy(q).cuda() for q in req[:n_plain]]
    S.ktau_query(kdb, qdev[0], k, ws, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in qdev:
        S.ktau_query(kdb, q, k, ws, stream=stream, check=False)
        stream.synchronize()
    plain_s = time.perf_counter() - t0
    plain_rows = int(sum(q.shape[0] for q in qdev))

    srv = S.KtauServer(kdb)
    # closed loop: everything submitted at once
    n_sat = 256
    for q in req[:8]:
        srv.wait(srv.submit(q, k))
    t0 = time.perf_counter()
    tickets = [srv.submit(q, k) for q in req[:n_sat]]
    for t in tickets:
        st, _, _ = srv.wait(t)
        if st != K.KTAU_OK:
            raise RuntimeError(f"serving: request failed with {st}")
    sat_s = time.perf_counter() - t0
    sat_rows = int(sum(q.shape[0] for q in req[:n_sat]))
    r_sat = n_sat / sat_s

    def poisson(rate: float, seed: int) -> dict:
        count = int(min(2000, max(100, rate * seconds)))
        arrivals, _ = synth.poisson_requests(count, rate, seed)
        order = [int(i) for i in rng.integers(0, len(req), count)]
        tick = [None] * count
        lat = [None] * count
        t_start = time.perf_counter()

        def submitter():
            for i in range(count):
                delay = t_start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tick[i] = srv.submit(req[order[i]], k)

        th = threading.Thread(target=submitter)
        th.start()
        for i in range(count):
            while tick[i] is None:
                time.sleep(0.0002)
            st, _, l = srv.wait(tick[i])
            if st != K.KTAU_OK:
                raise RuntimeError(f"serving: request failed with {st}")
            lat[i] = l
        th.join()
        wall = time.perf_counter() - t_start
        tot = np.array([x["total_us"] for x in lat]) / 1e3
        rows = sum(req[o].shape[0] for o in order)
        return {"rate_rps": rate, "requests": count, "p50_ms": float(np.percentile(tot, 50)),
                "p99_ms": float(np.percentile(tot, 99)), "mean_ms": float(tot.mean()),
                "pairs_per_s": rows * m / wall,
                "mean_batch_requests": float(np.mean([x["batch_requests"] for x in lat]))}

    rates = [poisson(0.5 * r_sat, 57), poisson(0.8 * r_sat, 58)]
    stats = srv.stats()
    srv.close()
    kdb.close()
    return {"workload": "database 20000 x 800 log-normal (seed 5), requests of U{1..64} query "
                        "rows (half near a database row), top-100 by |tau_B|, Poisson arrivals",
            "plain_per_request_pairs_per_s": plain_rows * m / plain_s,
            "plain_ms_per_request": plain_s * 1e3 / n_plain,
            "saturation_rps": r_sat, "saturation_pairs_per_s": sat_rows * m / sat_s,
            "at_rates": rates, "server": stats}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scheme", default=None, help="force a pair scheme (name or id)")
    ap.add_argument("--q", type=int, default=0, help="tile edge (default: the library's plain default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--plain-only", action="store_true", help="time only the plain form")
    ap.add_argument("--no-medium", action="store_true",
                    help="skip the medium workload (4096 x 512)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-batch comparison (256 matrices)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip the gene-vs-gene and sample-vs-sample shapes")
    ap.add_argument("--no-perm", action="store_true", help="skip the permutation test")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the short-row (naive count vs network) timing")
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="target length of each Poisson run")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the measurement, copy this many MiB device to device once "
                         "(a plain copy kernel of known size to scale HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1704_03767_amd import ktau as K
    from paper_1704_03767_amd import synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    X = synth.config_matrix(3)
    m, n = X.shape
    P = m * (m - 1) // 2
    Xd = torch.from_numpy(X).cuda()
    out_plain = K.alloc_outputs(P, m, Xd.device)
    out = K.alloc_outputs(P, m, Xd.device)       # the batched form's
    ws = K.alloc_workspace(m, n, Xd.device)
    stream = torch.cuda.current_stream()
    scheme = K.scheme_id(args.scheme) if args.scheme is not None else K.ktau_default_scheme(n)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        K.ktau_prepare(Xd, ws, out_plain["n1"], stream=stream)
        if ev is not None:
            ev[1].record(stream)
        K.ktau_pairs(m, n, out_plain, ws, scheme=scheme, q=args.q, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if K.ktau_status(ws) != K.KTAU_OK:
        raise RuntimeError("device reported an error in warm-up")
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = K.ktau_status(ws)
    if st != K.KTAU_OK:
        raise RuntimeError(f"device status {st}")
    ms_plain = (t1 - t0) * 1e3 / args.steps
    prep_all = [e[0].elapsed_time(e[1]) for e in events]
    pair_all = [e[1].elapsed_time(e[2]) for e in events]
    prep_ms = float(np.mean(prep_all))
    pair_ms = float(np.mean(pair_all))

    # the batched form of the same workload: a one-matrix plan (persistent
    # kernel, autotuned scheme, hipGraph), writing the same output arrays
    batched = None
    if not args.plain_only:
        plan = K.KtauBatch([Xd], outs=[out], stream=stream)
        for _ in range(max(1, args.warmup)):
            plan.run(stream)
        torch.cuda.synchronize()
        if plan.status(stream) != K.KTAU_OK:
            raise RuntimeError("batched warm-up failed")
        bev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)]
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            bev[i][0].record(stream)
            plan.run(stream)
            bev[i][1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if plan.status(stream) != K.KTAU_OK:
            raise RuntimeError("batched run failed")
        ms_batched = (t1 - t0) * 1e3 / args.steps
        step_all = [e[0].elapsed_time(e[1]) for e in bev]
        batched = {"ms_per_step": ms_batched, "pairs_per_s": P / (ms_batched * 1e-3),
                   "step_ms_median": float(np.median(step_all)),
                   "step_ms_min": float(np.min(step_all)),
                   "scheme": plan.plan(0)[0], "q": plan.plan(0)[1],
                   "equals_plain": outputs_equal(out, out_plain)}
        plan.close()
    else:
        out = out_plain
    ms_step = ms_plain if batched is None else batched["ms_per_step"]

    # the library's probes measure the int32 VALU and LDS peaks on this GPU
    probes = K.probe_peaks(stream=stream)
    steps_per_pair = merge_steps(n)
    ops_per_launch = P * steps_per_pair
    achieved = ops_per_launch / (pair_ms * 1e-3)
    src_hash = kernel_source_hash()
    kernel_tag = f"pairs_{K.ktau_scheme_names()[scheme]}_m{m}_n{n}"
    traffic = read_traffic(kernel_tag, src_hash)

    result = {
        "metric": METRIC,
        "value": P / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "allpairs m=16384 n=1024 log-normal, blocks of 64 rows at rho=0.6, "
                        "2% exact zeros, seed 3",
            "m": m, "n": n, "pairs": P, "form": "plain" if batched is None else "batched",
            "input_sha256": synth.sha256(X)[:16],
        },
        "plain": {"ms_per_step": ms_plain, "pairs_per_s": P / (ms_plain * 1e-3),
                  "scheme": K.ktau_scheme_names()[scheme], "q": args.q or K.ktau_plain_default_q(m, n),
                  "prepass_ms": prep_ms, "pair_kernel_ms": pair_ms,
                  "pair_kernel_ms_median": float(np.median(pair_all)),
                  "pair_kernel_ms_min": float(np.min(pair_all)),
                  "prepass_ms_median": float(np.median(prep_all))},
        "batched": batched,
        "probes": {"valu_lane_ops_per_s": probes["valu_lane_ops_per_s"],
                   "valu_published": INT_VALU_OPS,
                   "lds_bytes_per_s": probes["lds_bytes_per_s"],
                   "lds_reference_128B_per_clk": LDS_BYTES_PER_S,
                   "issue_per_simd_cycle": {
                       k: v / (1024 * 2.4e9) for k, v in probes["issue_wave_instr_per_s"].items()},
                   "note": "the VALU probe issues 16 v_add_u32 per iteration (ISA); its rate "
                           "is a denominator only where it does not exceed 256 CUs x 64 "
                           "lanes x 2.4 GHz; issue_per_simd_cycle: wave instructions per "
                           "SIMD and cycle at 2.4 GHz of each kind (0.25 = one per 4 cycles)"},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": INT_VALU_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved / INT_VALU_OPS,
            "traffic": traffic,
            "kernel": kernel_tag,
            "ops_per_pair": steps_per_pair,
            "source_hash": src_hash,
        },
    }
    if probes["valu_lane_ops_per_s"] <= INT_VALU_OPS:
        result["roofline"]["measured_peak"] = probes["valu_lane_ops_per_s"] / 1e12
        result["roofline"]["frac_of_measured"] = achieved / probes["valu_lane_ops_per_s"]
    if not args.no_medium:
        result["medium"] = medium(K, synth, torch, stream, max(5, args.steps))
    if not args.no_uneven:
        result["uneven_batch"] = uneven_batch(K, synth, torch, stream, max(2, args.steps))
    if not args.no_shapes:
        result["shapes"] = other_shapes(K, synth, torch, stream, max(2, args.steps))
        result["large_n"] = large_n(K, synth, torch, stream, max(2, args.steps))
    if not args.no_perm:
        result["perm_test"] = perm_test(K, synth, torch, stream, 2)
    if not args.no_small:
        result["small_n"] = small_n(K, synth, torch, stream, 5)
    if not args.no_serve:
        result["serving"] = serving(K, synth, torch, stream, args.serve_seconds)
        rates = result["serving"]["at_rates"]
        result["p50_ms"] = rates[-1]["p50_ms"]
        result["p99_ms"] = rates[-1]["p99_ms"]
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(X, args.cpu_seconds, gpu=out)
    print(json.dumps(result), flush=True)
    if args.copy_calibration_mib > 0:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
