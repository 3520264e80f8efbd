"""Throughput benchmark of the MI355X queues (one GPU).

Workload (the throughput sweep's headline point): a queue of capacity 2^20
with uint64 payloads, prefilled to n/2 outside the timed region; one step is
2^26 operation attempts by 2048 workgroups x 256 lanes (128 per lane), each op
an enqueue or a dequeue with probability 1/2 drawn from the seeded SplitMix64
stream, tried once.  Throughput = (successful enqueues + successful dequeues)
/ time (the paper's successful-operation throughput, Section V-A).  The
queue is not reset between steps: at a 50/50 mix its size stays near n/2.

Prints one JSON line.  Also measured in the same run: the atomic/bandwidth
roofline probes (same-address FAA rate, distinct-line CAS rate, HBM copy
bandwidth) and the CPU baselines (the oracle's sequential replay of the same
operation stream, and a host mutex-protected ring on all host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CAP = 1 << 20
LANES = 2048 * 256
OPS_PER_LANE = 128          # 2^26 attempts per step
STEP_OPS = LANES * OPS_PER_LANE
ITEM_BYTES = 8
# Algorithmic bytes per successful operation of the outer queue's fast path:
# two slot RMWs (8 B each, counted read + write), two slot loads, two
# threshold loads, one payload access (see the design notes).
BYTES_PER_OP = 2 * 16 + 2 * 8 + 2 * 8 + ITEM_BYTES
# G-WFQ-YMC has no index rings: one cell RMW (16 B) and about one more cell
# word access (the claim on dequeue, the value check on enqueue) per
# successful operation, on 32-byte cells.
BYTES_PER_OP_KIND = {"lfq": BYTES_PER_OP, "wfq": BYTES_PER_OP, "ymc": 32}
# Atomic read-modify-writes per successful operation at a 50/50 mix (the
# coalesced RMW rate is the bound once tickets are aggregated).  Ring queues:
# an enqueue consumes a free index (XOR), exchanges the payload and installs
# the index (CAS); a dequeue consumes the index (XOR), loads the payload and
# installs the index back into the free ring (CAS): (3 + 2) / 2.  YMC: an
# enqueue CASes the cell value, a dequeue loads it and claims the cell (CAS).
RMW_PER_OP_KIND = {"lfq": 2.5, "wfq": 2.5, "ymc": 1.0}
HBM_PEAK_GBS = 8000.0

# Scaled FETCH_SIZE + WRITE_SIZE bytes per launch of the timed kernel, from the
# two rocprofv3 --pmc runs summarised in the named profile; reported only while
# the kernel sources hash to the value they had when the counters were taken.
KERNEL_SOURCES = ("include/gq/common.h",
                  "include/gq/lfq.h",
                  "include/gq/wfq.h",
                  "include/gq/ymc.h",
                  "paper_2606_01693_amd/csrc/gq_lib.hip",
                  "include/gq.h", "include/gq_device.h")
_PROFILE = "profiles/k_mix_group_mixed5050_cap2p20_ops2p26.md"
TRAFFIC_PROFILE = {  # kind -> scaled FETCH_SIZE + WRITE_SIZE bytes per launch of the step kernel
    "lfq": {"sources_sha256_16": "bcb9e9c92146aba6", "bytes_per_launch": 3.697e9,
            "profile": _PROFILE},
    "wfq": {"sources_sha256_16": "bcb9e9c92146aba6", "bytes_per_launch": 3.799e9,
            "profile": _PROFILE},
    "ymc": {"sources_sha256_16": "bcb9e9c92146aba6", "bytes_per_launch": 3.053e9,
            "profile": _PROFILE},
}
NAMES = {"lfq": "G-LFQ", "wfq": "G-WFQ", "ymc": "G-WFQ-YMC"}
# The paper's per-operation profile metrics (VALU/op, WAIT/op) and L2 atomic
# requests per operation of the step kernels, from the rocprofv3 SQ_* and
# TCC_ATOMIC_sum runs summarised in the named profile; reported under the
# same conditions as the traffic figure.
_COUNTERS = "profiles/k_mix_group_mixed5050_sq_tcc_counters.md"
COUNTER_PROFILE = {
    "lfq": {"valu_per_op": 3.77, "wait_frac": 0.823, "wait_per_op": 1.23e-8,
            "tcc_atomic_per_op": 0.531},
    "wfq": {"valu_per_op": 5.31, "wait_frac": 0.774, "wait_per_op": 1.15e-8,
            "tcc_atomic_per_op": 0.529},
    "ymc": {"valu_per_op": 2.37, "wait_frac": 0.858, "wait_per_op": 1.28e-8,
            "tcc_atomic_per_op": 0.275},
}
COUNTER_SOURCES_HASH = "bcb9e9c92146aba6"


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_probes(gq, torch):
    """Roofline probes: R_ctr (same-address FAA), R_slot (distinct-line CAS),
    HBM copy bandwidth.  Each is timed with events on the current stream."""
    res = {}
    ctr = torch.zeros(64, dtype=torch.int64, device="cuda")

    def timed(fn, reps=3):
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return best

    lanes, iters = 2048 * 256, 64
    gq.probe_faa(ctr, lanes, 4, False)
    ms = timed(lambda: gq.probe_faa(ctr, lanes, iters, False))
    res["r_ctr_wave_faa_per_s"] = (lanes // 64) * iters / (ms * 1e-3)
    ms = timed(lambda: gq.probe_faa(ctr, 256 * 256, 16, True))
    res["r_ctr_lane_faa_per_s"] = 256 * 256 * 16 / (ms * 1e-3)
    # distinct-line CAS: one 8-byte slot per 128-byte line, as the remapped
    # ring places consecutive tickets
    nslots = 2 * CAP
    slots = torch.zeros(nslots * 16, dtype=torch.int64, device="cuda")
    # (64 CASes per lane, best of 5: a launch of a few tens of microseconds
    # measured the ramp-up and tail as much as the rate)
    gq.probe_cas(slots, nslots, 128, lanes, 2)
    ms = timed(lambda: gq.probe_cas(slots, nslots, 128, lanes, 64), reps=5)
    res["r_slot_cas_per_s"] = lanes * 64 / (ms * 1e-3)
    # linear slots: the consecutive tickets of a wavefront share lines
    gq.probe_cas(slots, nslots, 8, lanes, 2)
    ms = timed(lambda: gq.probe_cas(slots, nslots, 8, lanes, 64), reps=5)
    res["r_slot_cas_linear_per_s"] = lanes * 64 / (ms * 1e-3)
    del slots
    n = 1 << 28  # 2 GiB per buffer
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    gq.probe_copy(dst, src, n)
    ms = timed(lambda: gq.probe_copy(dst, src, n))
    res["hbm_copy_gbs"] = 2 * n * 8 / (ms * 1e-3) / 1e9
    del src, dst
    return res


def cpu_baselines(seed, sample_lanes, ops_per_lane=OPS_PER_LANE):
    """Oracle replay (1 core) of the headline step's op stream (its lanes x
    ops draws), and the host locked queue on all host cores."""
    import oracle
    import workloads
    roles = workloads.mix_roles(seed, sample_lanes, ops_per_lane)
    toks = workloads.mix_tokens(roles)
    pre = np.arange(1, CAP // 2 + 1, dtype=np.uint64) | np.uint64(0xFFFFFFFF << 32)
    t0 = time.perf_counter()
    st, _, _ = oracle.fifo_replay(roles.ravel(), toks.ravel(), capacity=CAP, prefill=pre)
    dt = time.perf_counter() - t0
    ok = int((st == 0).sum())
    replay = {"value": ok / dt / 1e6, "unit": "Mops/s", "cores": 1, "kind": "oracle",
              "sample": f"sequential FIFO replay of {sample_lanes} lanes x {ops_per_lane} ops "
                        f"of the same 50/50 stream in lane-major order, capacity 2^20, "
                        f"prefill n/2 ({roles.size} ops, {dt:.2f} s)"}
    cores = os.cpu_count() or 1
    threads = min(cores, 64)
    lroles = workloads.mix_roles(seed + 1, threads, 1 << 18)
    oke, okd, sec = oracle.locked_queue_run(lroles, CAP, CAP // 2)
    locked = {"value": (oke + okd) / sec / 1e6, "unit": "Mops/s", "cores": threads,
              "kind": "host mutex + ring",
              "sample": f"{threads} threads x 2^18 ops, 50/50 mix, capacity 2^20, prefill n/2"}
    return replay, locked


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


BFS_LANES = {"rmat22_ef16": (8192, 32768, 131072), "grid4096": (2048, 8192, 32768)}
# Algorithmic bytes of the queue BFS: per scanned adjacency entry a 4-byte
# column index and a 4-byte level probe; per reached vertex its two offsets,
# one enqueue and one dequeue of the outer queue (64 + 4 bytes each: slot
# RMWs, slot and threshold loads, the 4-byte payload) and its level CAS.
BFS_BYTES_PER_ENTRY = 8
BFS_BYTES_PER_VERTEX = 8 + 2 * (64 + 4) + 4


def bench_bfs(gq, torch, kinds=("lfq", "wfq", "ymc"), runs=3):
    """Queue-driven BFS GTEPS on the R-MAT scale-22 and 4096^2 grid inputs.
    GTEPS = (sum of degrees of reached vertices / 2) / time (undirected edges
    of the traversed component per second).  Levels are compared with the
    CPU BFS (oracle O7), which is also timed as the 1-core baseline."""
    import oracle
    import workloads
    out = {}
    seed = workloads.run_seed(4, 0)
    t0 = time.perf_counter()
    graphs = {"rmat22_ef16": workloads.rmat_graph(22, 16, seed=seed),
              "grid4096": workloads.grid_graph(4096, 4096)}
    log(f"[bench] graphs built in {time.perf_counter() - t0:.1f} s")
    roots = {"rmat22_ef16": workloads.bfs_root(graphs["rmat22_ef16"][0], seed),
             "grid4096": int(np.random.default_rng(workloads.run_seed(4, 1)).integers(0, 4096 ** 2))}
    for name, (off, cols) in graphs.items():
        nv = len(off) - 1
        root = roots[name]
        c0 = time.perf_counter()
        exp, nl, scanned = oracle.bfs(off, cols, root)
        cpu_s = time.perf_counter() - c0
        reached = int((exp != np.uint32(0xFFFFFFFF)).sum())
        log(f"[bench] cpu bfs {name}: {cpu_s * 1e3:.1f} ms, {nl} levels")
        edges = scanned / 2
        d_off = torch.tensor(off.astype(np.int32), device="cuda")
        d_cols = torch.tensor(cols.astype(np.int32), device="cuda")
        level = torch.empty(nv, dtype=torch.int32, device="cuda")
        ctl = torch.zeros(gq.bfs_ctl_bytes(len(cols)) // 8, dtype=torch.int64, device="cuda")
        cap = 1 << int(np.ceil(np.log2(nv)))
        res = {"vertices": nv, "reached": reached, "csr_entries": int(len(cols)), "root": root,
               "levels": nl, "bytes_model": f"{BFS_BYTES_PER_ENTRY} B per scanned entry + "
                                            f"{BFS_BYTES_PER_VERTEX} B per reached vertex",
               "edges_traversed": int(edges), "cpu_bfs_gteps": edges / cpu_s / 1e9,
               "cpu_bfs_ms": cpu_s * 1e3, "runs": {}}
        best = None
        for kind in kinds:
            for lanes in BFS_LANES[name]:
                # G-WFQ-YMC takes one pool cell per enqueue and per dequeue
                # attempt (each lane's last attempt of a level answers EMPTY)
                cells = (4 * nv + (nl + 4) * lanes * 4 + (1 << 16)) if kind == "ymc" else 0
                try:
                    qa = gq.Queue(kind, cap, item_width=4, max_threads=lanes, ymc_pool_cells=cells)
                    qb = gq.Queue(kind, cap, item_width=4, max_threads=lanes, ymc_pool_cells=cells)
                except gq.GQError as e:
                    log(f"[bench] bfs {name} {kind} lanes={lanes}: {e}")
                    continue
                ms = []
                ok = True
                for r in range(runs + 1):
                    qa.reset()
                    qb.reset()
                    e0, e1 = _events(torch)
                    e0.record()
                    try:
                        gq.bfs(qa, qb, d_off, d_cols, root, level, lanes, 256, ctl)
                    except gq.GQError as e:
                        log(f"[bench] bfs {name} {kind} lanes={lanes}: {e}")
                        ok = False
                        break
                    e1.record()
                    torch.cuda.synchronize()
                    log(f"[bench] bfs {name} {kind} lanes={lanes} run {r}: "
                        f"{e0.elapsed_time(e1):.2f} ms")
                    if r:
                        ms.append(e0.elapsed_time(e1))
                key = f"{gq_name(kind)} lanes={lanes}"
                err = qa.check_error()
                if not ok or err != gq.GQ_OK:
                    res["runs"][key] = {"error": gq.status_str(err) if err else "launch refused"}
                    qa.close()
                    qb.close()
                    continue
                match = bool(np.array_equal(level.cpu().numpy().view(np.uint32), exp))
                med = float(np.median(ms))
                nbytes = BFS_BYTES_PER_ENTRY * scanned + BFS_BYTES_PER_VERTEX * reached
                res["runs"][key] = {"ms_median": med, "gteps": edges / (med * 1e-3) / 1e9,
                                    "levels_match_oracle": match,
                                    "model_gbs": nbytes / (med * 1e-3) / 1e9,
                                    "hbm_frac": nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS}
                log(f"[bench] bfs {name} {key}: {med:.2f} ms, match={match}")
                if match and (best is None or med < best[1]):
                    best = (key, med)
                qa.close()
                qb.close()
        if best:
            res["best"] = {"config": best[0], "ms": best[1],
                           "gteps": edges / (best[1] * 1e-3) / 1e9}
        out[name] = res
    return out


def gq_name(kind):
    return NAMES[kind]


def bench_multi(gq, torch, kind="lfq", nq=256, ops=16, reps=5):
    """Many independent queues: 256 queues, capacities 2^e with e uniform in
    8..16 (seeded), each given one wavefront per 256 slots (at least one)
    and 16 operations per lane, i.e. 4n operations per queue, in a 50/50 mix.
    Compared: one launch for all queues, that launch replayed from a hipGraph,
    and one launch per queue (the plain single-queue driver)."""
    import workloads
    rng = np.random.default_rng(workloads.run_seed(5, 0))
    caps = [int(2 ** e) for e in rng.integers(8, 17, size=nq)]
    lanes = [64 * max(1, c // 256) for c in caps]
    pad = (-sum(lanes)) % 256
    lanes[int(np.argmax(caps))] += pad
    qs = [gq.Queue(kind, c, item_width=8, max_threads=l) for c, l in zip(caps, lanes)]
    pre_items = []
    for q, c in zip(qs, caps):
        t = torch.arange(1, c // 2 + 1, dtype=torch.int64, device="cuda") | (0xFFFFFFFF << 32)
        q.enqueue_batch(t)
        pre_items.append(t)
    m = gq.Multi(qs, lanes, block=256)
    counts = torch.zeros(8 * nq, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    total_ops = sum(lanes) * ops
    res = {"queues": nq, "capacities_log2_range": [8, 16], "total_lanes": sum(lanes),
           "ops_per_step": total_ops, "kind": NAMES[kind]}
    seed = workloads.run_seed(5, 10)
    torch.cuda.synchronize()  # prefill ran on the default stream

    def ok_count():
        c = counts.cpu().numpy().reshape(-1, 8)
        return int(c[:, 0].sum() + c[:, 1].sum())

    with torch.cuda.stream(s):
        m.run_mix(seed, ops, counts, stream=s)  # warmup
        s.synchronize()
        counts.zero_()
        s.synchronize()
        e0, e1 = _events(torch)
        e0.record(s)
        for r in range(reps):
            m.run_mix(seed + r, ops, counts, stream=s)
        e1.record(s)
        s.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res["one_launch"] = {"ms_per_step": ms, "mops": ok_count() / reps / (ms * 1e-3) / 1e6}
        counts.zero_()
        m.capture(seed + 100, ops, counts, s)
        m.replay(s)
        s.synchronize()
        counts.zero_()
        s.synchronize()
        e0, e1 = _events(torch)
        e0.record(s)
        for r in range(reps):
            m.replay(s)
        e1.record(s)
        s.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res["graph_replay"] = {"ms_per_step": ms, "mops": ok_count() / reps / (ms * 1e-3) / 1e6}
        counts.zero_()
        s.synchronize()
        e0, e1 = _events(torch)
        e0.record(s)
        for r in range(reps):
            for i, q in enumerate(qs):
                q.run_mix(seed + 1000 + r, lanes[i], ops, counts[8 * i:8 * i + 8], stream=s)
        e1.record(s)
        s.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res["launch_per_queue"] = {"ms_per_step": ms,
                                   "mops": ok_count() / reps / (ms * 1e-3) / 1e6}
    for q in qs:
        if q.check_error() != gq.GQ_OK:
            res["error"] = gq.status_str(q.check_error())
    res["speedup_graph_vs_per_queue"] = (res["graph_replay"]["mops"] /
                                         res["launch_per_queue"]["mops"])
    m.close()
    for q in qs:
        q.close()
    # the autotuner's lane allotment for the same queues and work per queue
    from paper_2606_01693_amd import autotune
    t = autotune.tune_multi(kind, caps, waves_per_256_slots=(0.5, 1, 2, 4), ops_factor=4, reps=3)
    res["autotuned"] = {"waves_per_256_slots": t.best["waves_per_256_slots"],
                        "ms_per_step": t.best_ms, "mops": t.best_mops,
                        "table": [{k: v for k, v in row.items()} for row in t.table]}
    return res


def bench_ticket_ablation(gq, torch, kinds, seed, args, reps=3):
    """The step's kernel with each ticket grouping: 64 lanes (every wavefront
    takes its own tickets, WaveFAA alone) up to 1024 lanes (one FAA per
    counter per workgroup).  Same workload; median kernel time of `reps`
    launches after one warmup."""
    out = {}
    for kind in kinds:
        for tg in (64, 256, 1024):
            q = gq.Queue(kind, CAP, item_width=ITEM_BYTES, max_threads=LANES,
                         slot_mode=args.slot_mode, fenced=args.fenced,
                         ymc_pool_cells=(1 << 28) if kind == "ymc" else 0, ticket_group=tg)
            pre = torch.arange(1, CAP // 2 + 1, dtype=torch.int64, device="cuda") | (0xFFFFFFFF << 32)
            q.enqueue_batch(pre)
            counts = torch.zeros(8, dtype=torch.int64, device="cuda")
            ms = []
            for r in range(reps + 1):
                e0, e1 = _events(torch)
                e0.record()
                q.run_mix(seed + 500 + r, LANES, OPS_PER_LANE, counts)
                e1.record()
                torch.cuda.synchronize()
                if r:
                    ms.append(e0.elapsed_time(e1))
            c = counts.cpu().tolist()
            ok = (c[0] + c[1]) / (reps + 1)
            med = float(np.median(ms))
            assert q.check_error() == gq.GQ_OK
            out[f"{NAMES[kind]} group={tg}"] = {
                "kernel_ms": med, "mops": ok / (med * 1e-3) / 1e6,
                "launch": (f"{LANES // 256} WGs x 256 lanes, per-wavefront tickets" if tg == 64
                           else f"{LANES // tg} WGs x {tg} lanes, one ticket FAA per WG")}
            log(f"[bench] tickets {NAMES[kind]} group={tg}: {med:.2f} ms, "
                f"{ok / (med * 1e-3) / 1e6:.0f} Mops/s")
            q.close()
            del pre
            torch.cuda.empty_cache()
    return out


def serve_level_hash(levels: np.ndarray, seed: int) -> int:
    """The serving checksum: wrapping sum of splitmix64(seed, v) * (level[v] + 1)."""
    import workloads
    v = np.arange(len(levels), dtype=np.uint64)
    with np.errstate(over="ignore"):
        w = workloads.splitmix64(seed, v)
        return int((w * (levels.astype(np.uint64) + np.uint64(1))).sum(dtype=np.uint64))


RT_SIZE = (1920, 1080)
RT_LANES = (1 << 9, 1 << 11, 1 << 13, 1 << 15)


def bench_rt(gq, torch, reps=5):
    """Tile-based wavefront ray tracing (1920 x 1080, 32 x 32 tiles): MRays/s
    = path segments traced / render time (median of `reps` after a warmup),
    for per-tile G-LFQ and G-WFQ queues and for stream compaction, at lane
    counts 2^9 .. 2^15.  Every image is compared bit for bit with the
    compaction image of the same scene."""
    from workloads import scenes
    w, h = RT_SIZE
    out = {}
    for name in ("complex", "cornell"):
        sc = (scenes.complex_scene(20260601, w, h) if name == "complex"
              else scenes.cornell_scene(w, h))
        res, ref_img = {}, None
        for method, kind in (("compact", "lfq"), ("G-LFQ", "lfq"), ("G-WFQ", "wfq")):
            for lanes in RT_LANES:
                r = gq.RayTracer(kind, w, h, tile=32, lanes=lanes)
                r.set_scene(sc)
                m = gq.RT_COMPACT if method == "compact" else gq.RT_QUEUES
                img, segs, stats = r.render(m)
                ms = []
                for _ in range(reps):
                    e0, e1 = _events(torch)
                    e0.record()
                    r.render(m, img, segs, stats)
                    e1.record()
                    torch.cuda.synchronize()
                    ms.append(e0.elapsed_time(e1))
                err = r.check_error()
                st = stats.cpu().tolist()
                bits = img.cpu().numpy().view(np.uint32)
                if ref_img is None:
                    ref_img = bits.copy()
                med = float(np.median(ms))
                res[f"{method} lanes={lanes}"] = {
                    "ms": med, "mrays_s": st[0] / (med * 1e-3) / 1e6, "segments": st[0],
                    "empty_polls": st[2], "ok": bool(err == 0 and np.array_equal(bits, ref_img))}
                log(f"[bench] rt {name} {method} lanes={lanes}: {med:.2f} ms, "
                    f"{res[f'{method} lanes={lanes}']['mrays_s']:.0f} MRays/s, ok={err == 0}")
                r.close()
        best_c = max(v["mrays_s"] for k, v in res.items() if k.startswith("compact"))
        same = {k: v["mrays_s"] / res["compact lanes=" + k.split("lanes=")[1]]["mrays_s"]
                for k, v in res.items()}
        out[name] = {"runs": res, "best_compact_mrays_s": best_c,
                     "relative_to_compact_same_lanes": same,
                     "relative_to_best_compact": {k: v["mrays_s"] / best_c for k, v in res.items()}}
    return out


def bench_serve(gq, torch, njobs=1000, pool_size=64, team_lanes=1024, budget=16 << 30):
    """Serving: a pool of 64 R-MAT graphs (scale uniform in 12..20, edge
    factor 16, seeded), 1000 BFS jobs each on a graph drawn from the pool,
    admitted by a 16 GiB device-memory budget.  The service rate is measured
    with every job arriving at once; then Poisson arrivals at 0.5 and 0.9 of
    that rate give latency percentiles (arrival to completion seen by the
    host).  Every job's level hash is compared with the CPU BFS's, in the mix
    and with each distinct job run alone."""
    import oracle
    import workloads
    seed = workloads.run_seed(5, 500)
    rng = np.random.default_rng(seed)
    scales = rng.integers(12, 21, size=pool_size)
    t0 = time.perf_counter()
    pool = []
    for i, sc in enumerate(scales):
        off, cols = workloads.rmat_graph(int(sc), 16, seed=seed + i)
        root = workloads.bfs_root(off, seed + 7 * i)
        exp, nl, _ = oracle.bfs(off, cols, root)
        pool.append({"off": torch.tensor(off.astype(np.int32), device="cuda"),
                     "cols": torch.tensor(cols.astype(np.int32), device="cuda"), "root": root,
                     "hash": serve_level_hash(exp, gq.SERVE_HASH_SEED), "scale": int(sc)})
    torch.cuda.synchronize()  # the graphs are resident before the server starts
    log(f"[bench] serve pool of {pool_size} graphs ready in {time.perf_counter() - t0:.1f} s")
    pick = rng.integers(0, pool_size, size=njobs)
    reqs = [(pool[i]["off"], pool[i]["cols"], pool[i]["root"]) for i in pick]
    want = np.array([pool[i]["hash"] for i in pick], dtype=np.uint64)
    teams = gq.device_info()["cus"]
    out = {"jobs": njobs, "pool": f"{pool_size} R-MAT graphs, scale 12..20, edge factor 16",
           "teams": teams, "team_lanes": team_lanes, "budget_gib": budget / 2**30,
           "job_queue": "G-LFQ", "per_job_queues": "G-LFQ"}
    ok = True
    with gq.Server(teams=teams, team_lanes=team_lanes, kind="lfq", budget_bytes=budget,
                   ring_slots=1024) as srv:
        sat = srv.run(reqs, np.zeros(njobs, dtype=np.int64))
        ok &= bool((sat["status"] == 0).all() and np.array_equal(sat["level_hash"], want))
        makespan = sat["done_ns"].max() / 1e9
        mu = njobs / makespan
        out["service_rate_jobs_s"] = mu
        log(f"[bench] serve saturation: {makespan * 1e3:.1f} ms for {njobs} jobs, "
            f"{mu:.0f} jobs/s, ok={ok}")
        for frac in (0.5, 0.9):
            gaps = rng.exponential(1e9 / (frac * mu), size=njobs)
            arr = np.cumsum(gaps).astype(np.int64)
            r = srv.run(reqs, arr)
            good = bool((r["status"] == 0).all() and np.array_equal(r["level_hash"], want))
            ok &= good
            lat = (r["done_ns"] - r["arrival_ns"]) / 1e6
            span = (r["done_ns"].max() - r["arrival_ns"].min()) / 1e9
            out[f"lambda_{frac}"] = {
                "arrival_rate_jobs_s": frac * mu, "jobs_s": njobs / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_device_ms": float(r["device_ns"].mean() / 1e6),
                "levels_match_oracle": good}
            log(f"[bench] serve lambda={frac}: {out[f'lambda_{frac}']}")
        alone = srv.run([(p["off"], p["cols"], p["root"]) for p in pool],
                        np.zeros(pool_size, dtype=np.int64), max_inflight=1)
        want_alone = np.array([p["hash"] for p in pool], dtype=np.uint64)
        out["alone_equals_oracle"] = bool((alone["status"] == 0).all() and
                                          np.array_equal(alone["level_hash"], want_alone))
    out["levels_match_oracle"] = ok
    return out


def bench_c2(gq, torch, kinds, seed, args):
    """The throughput sweep's other points: (a) the mixed 50/50 workload with
    2^26 attempts split over G x 256 lanes, G = 1, 2, 4, ..., 2048 (the lanes
    run in workgroups of min(ticket group, G x 256) lanes -- 1024 by default --
    each taking its first tickets with one FAA per counter; the queue is reset
    and prefilled to n/2 before each point); (b) 32 fill/drain rounds through
    the host batch API (enqueue a batch of n = 2^20 items, then dequeue a batch
    of n).  Kernel time by events."""
    out = {"mix_by_workgroups": {}, "fill_drain": {}}
    total = 1 << 26
    group = args.ticket_group or 1024
    for kind in kinds:
        q = gq.Queue(kind, CAP, item_width=ITEM_BYTES, max_threads=LANES,
                     ymc_pool_cells=(1 << 27) if kind == "ymc" else 0,
                     ticket_group=args.ticket_group)
        pre = torch.arange(1, CAP // 2 + 1, dtype=torch.int64, device="cuda") | (0xFFFFFFFF << 32)
        counts = torch.zeros(8, dtype=torch.int64, device="cuda")
        row = {}
        g = 1
        while g <= 2048:
            lanes = g * 256
            ops = total // lanes
            q.reset()
            q.enqueue_batch(pre)
            counts.zero_()
            e0, e1 = _events(torch)
            e0.record()
            q.run_mix(seed + 900 + g, lanes, ops, counts)
            e1.record()
            torch.cuda.synchronize()
            c = counts.cpu().tolist()
            ms = e0.elapsed_time(e1)
            wg = min(group, lanes) if group > 64 else 256
            row[f"{g}x256"] = {"ms": ms, "mops": (c[0] + c[1]) / (ms * 1e-3) / 1e6,
                               "launch": f"{lanes // wg} WGs x {wg} lanes"}
            g *= 2
        assert q.check_error() == gq.GQ_OK
        out["mix_by_workgroups"][NAMES[kind]] = row
        log(f"[bench] c2 sweep {NAMES[kind]}: " +
            ", ".join(f"G={k}: {v['mops']:.0f}" for k, v in row.items()))
        q.close()
        q = gq.Queue(kind, CAP, item_width=ITEM_BYTES, max_threads=LANES,
                     ymc_pool_cells=(1 << 27) if kind == "ymc" else 0,
                     ticket_group=args.ticket_group)
        items = torch.arange(1, CAP + 1, dtype=torch.int64, device="cuda")
        outb = torch.zeros(CAP, dtype=torch.int64, device="cuda")
        nok = torch.zeros(1, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record()
        for _ in range(32):
            q.enqueue_batch(items, num_ok=nok)
            q.dequeue_batch(outb, num_ok=nok)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ok = int(nok.item())
        good = ok == 64 * CAP and q.check_error() == gq.GQ_OK and \
            bool(torch.equal(outb.sort().values, items))
        out["fill_drain"][NAMES[kind]] = {"ms": ms, "mops": ok / (ms * 1e-3) / 1e6,
                                          "all_ok_and_last_round_conserved": good}
        log(f"[bench] c2 fill/drain {NAMES[kind]}: {ms:.2f} ms, {ok / (ms * 1e-3) / 1e6:.0f} "
            f"Mops/s, ok={good}")
        q.close()
        del pre, items, outb
        torch.cuda.empty_cache()
    return out


def bench_timed(gq, torch, kinds, reps=5, warmup_us=1000, window_us=5000):
    """The paper's micro-benchmark form: fixed-duration balanced and split
    kernels (producer fractions 25/50/75 %), T = 2^9 .. 2^15 lanes in
    workgroups of 256, per-wavefront tickets, capacity 2^20 prefilled to n/2;
    Mops/s = successful operations completed in the window / window, median
    of 5."""
    out = {}
    for kind in kinds:
        q = gq.Queue(kind, CAP, item_width=ITEM_BYTES, max_threads=1 << 15,
                     ymc_pool_cells=(1 << 28) if kind == "ymc" else 0)
        pre = torch.arange(1, CAP // 2 + 1, dtype=torch.int64, device="cuda") | (0xFFFFFFFF << 32)
        counts = torch.zeros(10, dtype=torch.int64, device="cuda")
        ctl = torch.zeros(4, dtype=torch.int64, device="cuda")
        modes = [("balanced", 50), ("split", 25), ("split", 50), ("split", 75)]
        res = {}
        for mode, pct in modes:
            key = "balanced" if mode == "balanced" else f"split{pct}"
            row = {}
            for lg in range(9, 16):
                vals = []
                for _ in range(reps):
                    q.reset()
                    q.enqueue_batch(pre)
                    counts.zero_()
                    q.run_timed(mode, 1 << lg, counts, ctl, prod_pct=pct, warmup_us=warmup_us,
                                window_us=window_us)
                    c = counts.cpu().tolist()
                    vals.append((c[0] + c[1]) / (window_us * 1e-6) / 1e6)
                row[str(1 << lg)] = float(np.median(vals))
            if q.check_error() != gq.GQ_OK:
                row["error"] = gq.status_str(q.check_error())
            res[key] = row
            log(f"[bench] timed {NAMES[kind]} {key}: " +
                ", ".join(f"{k}: {v:.0f}" for k, v in row.items() if k != "error"))
        out[NAMES[kind]] = res
        q.close()
        del pre
        torch.cuda.empty_cache()
    return out


def bench_c3(gq, torch, kinds=("lfq", "wfq", "ymc"), items=1 << 23, cap=1 << 16, waves=1024):
    """Imbalanced producer/consumer runs: 1024 wavefronts of which the seed
    makes 128, 512 or 896 producers; a lane is active in a round with
    probability 1, 1/2 or 1/64; producers retry on FULL, consumers on EMPTY,
    until 2^23 items went through.  Mops/s counts successful operations
    (2 x items) over the kernel time; conservation is checked through the
    driver's multiset checksums."""
    import workloads
    lanes = waves * 64
    out = {}
    for kind in kinds:
        q = gq.Queue(kind, cap, item_width=8, max_threads=lanes,
                     ymc_pool_cells=(1 << 31) if kind == "ymc" else 0)
        for prod in (128, 512, 896):
            for l2p in (0, 1, 6):
                seed = workloads.run_seed(3, prod + l2p)
                mask = workloads.producer_waves(seed, waves, prod)
                role = torch.tensor(np.repeat(np.where(mask, 0, 1), 64).astype(np.uint8),
                                    device="cuda")
                quota = -(-items // (prod * 64))
                target = quota * prod * 64
                counts = torch.zeros(8, dtype=torch.int64, device="cuda")
                q.reset()
                torch.cuda.synchronize()
                e0, e1 = _events(torch)
                e0.record()
                q.run_prodcons(seed, lanes, 256, role, quota, target, l2p, 0, counts,
                               max_rounds=1 << 30, time_limit_ms=30000)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                c = counts.cpu().numpy().view(np.uint64)
                ok = bool(c[0] == target and c[1] == target and c[4] == c[6] and c[5] == c[7]
                          and q.check_error() == gq.GQ_OK)
                key = f"{NAMES[kind]} {prod}:{waves - prod} p=2^-{l2p}"
                out[key] = {"ms": ms, "mops": 2 * target / (ms * 1e-3) / 1e6,
                            "full_retries": int(c[2]), "empty_retries": int(c[3]),
                            "conserved": ok}
                log(f"[bench] c3 {key}: {ms:.2f} ms, {out[key]['mops']:.0f} Mops/s, ok={ok}")
        q.close()
        torch.cuda.empty_cache()
    return out


# The step's headline queue: G-WFQ, the paper's wait-free queue (its first
# contribution).  G-LFQ and G-WFQ-YMC run the same step and are reported under
# "variants".
HEADLINE = "wfq"
# G-WFQ-YMC's cell pool: the queue is reset and prefilled before every step
# (outside the timed region), so the pool needs to hold one step's cells only:
# every attempt takes at most one T or H ticket on the fast path (a ticket is a
# cell), i.e. LANES * OPS_PER_LANE cells, plus the prefill's n/2, plus slow-path
# retries, far below 2^27 cells (3 GiB).
YMC_STEP_POOL = 1 << 27


def step_plan(steps: int, warmup: int) -> dict:
    """How the timed steps use the queues: every step starts from a freshly
    reset queue prefilled to n/2, so nothing a step needs grows with the
    number of steps (G-WFQ-YMC's pool in particular)."""
    need = LANES * OPS_PER_LANE + CAP // 2
    return {"launches": warmup + steps, "reset_each_step": True,
            "ymc_pool_cells": YMC_STEP_POOL, "ymc_cells_needed_per_step": need,
            "fits": need <= YMC_STEP_POOL}


def step_shape(gq, kind: str, ticket_group: int):
    """(lanes, ops per lane) of a variant's step: 2^26 attempts by the largest
    power-of-two number of lanes, at most 2^19, that the device holds at once
    in the group kernel's workgroups (one round of workgroups, none waiting
    for another to finish).  The per-wavefront form (ticket group 64) keeps
    2^19 lanes in workgroups of 256."""
    g = ticket_group or 1024
    if g <= 64:
        return LANES, OPS_PER_LANE
    resident = gq.resident_blocks("mix_group", kind, g) * g
    lanes = LANES
    while lanes > g and lanes > resident:
        lanes //= 2
    return lanes, STEP_OPS // lanes


def launch_desc(ticket_group: int, lanes: int = LANES) -> str:
    g = ticket_group or 1024
    if g <= 64:
        return f"{lanes // 256} WGs x 256 lanes, per-wavefront ticket FAAs"
    return f"{lanes // g} WGs x {g} lanes, one ticket FAA per counter per WG"


def checksums(v: np.ndarray):
    """(count, wrapping sum of v, wrapping sum of v*v) of uint64 items."""
    with np.errstate(over="ignore"):
        return (int(v.shape[0]), int(v.sum(dtype=np.uint64)), int((v * v).sum(dtype=np.uint64)))


def csum_add(a, b):
    m = (1 << 64) - 1
    return a[0] + b[0], (a[1] + b[1]) & m, (a[2] + b[2]) & m


def run_variant(gq, torch, kind, args, base_seed):
    """Warmup + timed steps of one queue variant.  Each step: reset the queue
    and prefill it to n/2 (untimed), synchronise, launch the mixed kernel
    (timed by wall clock with a synchronisation on both sides, and by HIP
    events on the launch stream), then drain what is left (untimed) and check
    conservation of the step with the kernel's multiset checksums: prefill +
    enqueued = dequeued + drained (counts and wrapping sums of v and v*v)."""
    lanes, ops = step_shape(gq, kind, args.ticket_group)
    q = gq.Queue(kind, CAP, item_width=ITEM_BYTES, max_threads=lanes,
                 slot_mode=args.slot_mode, fenced=args.fenced,
                 ymc_pool_cells=YMC_STEP_POOL if kind == "ymc" else 0,
                 ticket_group=args.ticket_group)
    try:
        pre = torch.arange(1, CAP // 2 + 1, dtype=torch.int64, device="cuda") | (0xFFFFFFFF << 32)
        pre_sums = checksums(pre.cpu().numpy().view(np.uint64))
        counts = torch.zeros(8, dtype=torch.int64, device="cuda")
        out = torch.zeros(CAP, dtype=torch.int64, device="cuda")
        ost = torch.zeros(CAP, dtype=torch.uint8, device="cuda")
        kms, walls, oks, conserved = [], [], [], True
        q.clear_stats()
        for i in range(args.warmup + args.steps):
            q.reset()
            q.enqueue_batch(pre)
            counts.zero_()
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            t0 = time.perf_counter()
            e0.record()
            q.run_mix(base_seed + i, lanes, ops, counts)
            e1.record()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            # untimed: drain the remainder and check the step's conservation
            q.dequeue_batch(out, ost)
            c = counts.cpu().numpy().view(np.uint64).tolist()
            st = ost.cpu().numpy()
            left = out.cpu().numpy().view(np.uint64)[st == gq.GQ_OK]
            put = csum_add(pre_sums, (c[0], c[6], c[7]))
            got = csum_add((c[1], c[4], c[5]), checksums(left))
            ok_step = put == got and c[0] + c[1] + c[2] + c[3] == STEP_OPS
            conserved &= ok_step
            if i >= args.warmup:
                kms.append(e0.elapsed_time(e1))
                walls.append((t1 - t0) * 1e3)
                oks.append(c[0] + c[1])
        err = q.check_error()
        st = q.stats()
        kms_a, walls_a = np.array(kms), np.array(walls)
        ok_mean = float(np.mean(oks))
        res = {
            "name": NAMES[kind],
            "kernel": (f"k_mix<{NAMES[kind]}>" if (args.ticket_group or 1024) <= 64
                       else "k_mix_group_lfq" if kind == "lfq"
                       else f"k_mix_group<{NAMES[kind]}>"),
            "launch": launch_desc(args.ticket_group, lanes),
            "lanes": lanes,
            "ops_per_lane": ops,
            "mops": sum(oks) / (walls_a.sum() * 1e-3) / 1e6,
            "mops_kernel": ok_mean / (float(np.median(kms_a)) * 1e-3) / 1e6,
            "ok_ops_per_step": ok_mean,
            "kernel_ms": {"median": float(np.median(kms_a)), "mean": float(kms_a.mean()),
                          "min": float(kms_a.min()), "max": float(kms_a.max()),
                          "per_step": [round(x, 4) for x in kms]},
            "step_wall_ms": {"median": float(np.median(walls_a)), "mean": float(walls_a.mean()),
                             "min": float(walls_a.min()), "max": float(walls_a.max())},
            "conserved_every_step": bool(conserved),
            "device_error": gq.status_str(err) if err else None,
            "dropped_ops": st.dropped,
            "cas_fail_per_ok_op": st.cas_fail / max(1, sum(oks)),
            "slow_path_entries_per_step": st.slow_enter / (args.warmup + args.steps),
            "helps_per_step": st.helps / (args.warmup + args.steps),
        }
        log(f"[bench] {kind}: kernel ms median {res['kernel_ms']['median']:.3f} "
            f"(min {res['kernel_ms']['min']:.3f}, max {res['kernel_ms']['max']:.3f}), "
            f"{res['mops']:.0f} Mops/s by wall clock, conserved={conserved}, err={err}")
        return res
    finally:
        q.close()


def section(out, key, fn):
    """Run one bench section; an exception is recorded, not fatal."""
    t0 = time.perf_counter()
    try:
        out[key] = fn()
    except Exception as e:  # noqa: BLE001 -- the JSON line must still be printed
        out[key] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] section {key} failed: {e}")
    out.setdefault("section_seconds", {})[key] = round(time.perf_counter() - t0, 1)
    log(f"[bench] section {key}: {out['section_seconds'][key]} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kinds", default="lfq,wfq,ymc",
                    help="comma-separated queue variants run by each step")
    ap.add_argument("--slot-mode", default="linear", choices=["remap", "padded", "linear"])
    ap.add_argument("--fenced", action="store_true",
                    help="release/acquire payload hand-off instead of the atomic exchange")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-probes", action="store_true")
    ap.add_argument("--no-bfs", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-rt", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-timed", action="store_true")
    ap.add_argument("--ticket-group", type=int, default=0,
                    help="lanes per ticket FAA in the step (64 = one wavefront; 0 = 1024)")
    ap.add_argument("--no-ablation", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_2606_01693_amd as gq
    import workloads

    torch.cuda.set_device(0)
    info = gq.device_info()
    log(f"[bench] device {info}")
    kinds = [k for k in args.kinds.split(",") if k]
    head = HEADLINE if HEADLINE in kinds else kinds[0]
    base_seed = workloads.run_seed(2, 0)
    plan = step_plan(args.steps, args.warmup)
    variants = {}
    for kind in kinds:
        try:
            variants[kind] = run_variant(gq, torch, kind, args, base_seed)
        except Exception as e:  # noqa: BLE001 -- report and go on with the other variants
            variants[kind] = {"name": NAMES[kind], "error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {kind} failed: {e}")
        torch.cuda.empty_cache()
    hv = variants[head]
    ok_head = "error" not in hv and hv["conserved_every_step"] and hv["device_error"] is None
    out = {
        "metric": "Mops/s enq+deq at 50/50 mix, 2^20-slot queue",
        "value": hv["mops"] if ok_head else None,
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hv["step_wall_ms"]["mean"] if "error" not in hv else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"{NAMES[head]}: mixed 50/50 enqueue/dequeue, capacity 2^20, uint64 "
                        f"payload, 2^26 op attempts per step by {hv.get('lanes', LANES)} lanes x "
                        f"{hv.get('ops_per_lane', OPS_PER_LANE)} ops "
                        f"({hv.get('launch', launch_desc(args.ticket_group))}; the most lanes, up "
                        f"to 2^19, resident at once), queue reset and prefilled to n/2 "
                        f"before each step (untimed); slots={args.slot_mode}, hand-off="
                        + ("fenced" if args.fenced else "atomic"),
            "queue": NAMES[head], "capacity": CAP, "lanes": hv.get("lanes", LANES),
            "ops_per_lane": hv.get("ops_per_lane", OPS_PER_LANE),
            "parallelism": "single GPU",
        },
        "step_plan": plan,
        "variants": variants,
    }
    if "error" not in hv:
        bpo = BYTES_PER_OP_KIND[head]
        kavg = hv["kernel_ms"]["mean"]
        achieved_gbs = hv["ok_ops_per_step"] * bpo / (kavg * 1e-3) / 1e9
        traffic = TRAFFIC_PROFILE.get(head)
        out["roofline"] = {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            # the profiled configuration only: default ticket group, linear
            # slots, atomic hand-off, unchanged kernel sources
            "traffic": (traffic["bytes_per_launch"] if traffic and
                        kernel_sources_hash() == traffic["sources_sha256_16"] and
                        args.ticket_group in (0, 1024) and args.slot_mode == "linear" and
                        not args.fenced else None),
            "kernel": hv["kernel"],
            "kernel_ms_avg": kavg,
            "bytes_per_ok_op": bpo,
            "ok_ops_per_launch": hv["ok_ops_per_step"],
        }
    if (kernel_sources_hash() == COUNTER_SOURCES_HASH and args.ticket_group in (0, 1024)
            and args.slot_mode == "linear" and not args.fenced):
        out["profile_counters"] = {NAMES[k]: COUNTER_PROFILE[k] for k in kinds}
        out["profile_counters"]["profile"] = _COUNTERS
    if not args.no_probes:
        def probes():
            p = measure_probes(gq, torch)
            # Each of the four ticket counters serves one of every two
            # operations (enqueues: fq.Head, aq.Tail; dequeues: aq.Head,
            # fq.Tail), and one ticket FAA covers the a lanes of a ticket group
            # taking the same branch (a = group / 2 at a 50/50 mix: 32 for one
            # wavefront, 512 for the default 1024-lane group).  Each successful
            # op performs RMW_PER_OP_KIND atomic RMWs at the layout's stride.
            group = args.ticket_group or 1024
            a = group / 2.0
            r_slot = p["r_slot_cas_linear_per_s" if args.slot_mode == "linear"
                       else "r_slot_cas_per_s"]
            per_kernel = {}
            for k in kinds:
                if "error" in variants[k]:
                    continue
                b = min(2 * a * p["r_ctr_wave_faa_per_s"], r_slot / RMW_PER_OP_KIND[k],
                        p["hbm_copy_gbs"] * 1e9 / BYTES_PER_OP_KIND[k])
                per_kernel[NAMES[k]] = {"bound_mops": b / 1e6,
                                        "frac": variants[k]["mops_kernel"] * 1e6 / b}
            return dict(p, ticket_group=group, lanes_per_faa=a, per_kernel=per_kernel)
        section(out, "atomic_roofline", probes)
    torch.cuda.empty_cache()
    if not args.no_ablation:
        section(out, "ticket_ablation",
                lambda: bench_ticket_ablation(gq, torch, kinds, base_seed, args))
    if not args.no_c2:
        section(out, "c2_sweep", lambda: bench_c2(gq, torch, kinds, base_seed, args))
    if not args.no_timed:
        section(out, "fixed_duration", lambda: bench_timed(gq, torch, kinds))
    if not args.no_multi:
        section(out, "batched_multi_queue", lambda: bench_multi(gq, torch))
    if not args.no_c3:
        def c3():
            r = bench_c3(gq, torch)
            from paper_2606_01693_amd import autotune
            t = autotune.tune_prodcons("wfq", prod_waves=128, log2_inv_p=1,
                                       patience_options=((16, 64), (64, 256), (256, 1024)),
                                       help_delays=(64,), time_limit_ms=5000)
            r["wfq_patience_tuning_128_896_p_half"] = {"best": t.best, "best_ms": t.best_ms,
                                                       "table": t.table}
            return r
        section(out, "imbalanced_prodcons", c3)
    if not args.no_bfs:
        section(out, "bfs", lambda: bench_bfs(gq, torch))
    if not args.no_serve:
        section(out, "serve", lambda: bench_serve(gq, torch))
    if not args.no_rt:
        section(out, "raytrace", lambda: bench_rt(gq, torch))
    if not args.no_cpu:
        def cpu():
            hv = out["variants"].get(head, {})
            replay, locked = cpu_baselines(base_seed, hv.get("lanes", LANES),
                                           hv.get("ops_per_lane", OPS_PER_LANE))
            out["cpu_baseline"] = replay
            out["host"] = {"cpu": platform.processor() or platform.machine(),
                           "cores": os.cpu_count()}
            return locked
        section(out, "cpu_locked_queue", cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
