"""GPU parity tests: the HIP queues, called through the C ABI, against the CPU
oracle.  A concurrent queue has many correct outcomes, so parity means: the
recorded history passes the oracle's checks (exact multiset conservation,
per-producer order, violation scan, exhaustive linearizability on tiny runs),
and deterministic shapes (one lane; one wavefront into a quiescent queue;
stream-ordered batches) match the sequential FIFO replay exactly."""
import random

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import prefill, assert_clean, check_history, drain_fifo, history, torch, u64

pytestmark = pytest.mark.gpu

KINDS = ["lfq", "wfq", "ymc"]
BOUNDED = {"lfq": True, "wfq": True, "ymc": False}


def make_queue(kind, n, width=8, lanes=1024, slot_mode="linear", **opts):
    import paper_2606_01693_amd as gq
    print(f"[case] kind={kind} n={n} width={width} lanes={lanes} slots={slot_mode} {opts}",
          flush=True)
    return gq.Queue(kind, n, item_width=width, max_threads=lanes, slot_mode=slot_mode, **opts)


def cap_of(kind, n):
    return n if BOUNDED[kind] else 0


def all_zero(rep):
    return all(v == 0 for v in rep.values())


# ---------------------------------------------------------------------------
# Deterministic shapes: exact equality with the sequential replay
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n,seed", [(2, 0), (4, 1), (16, 2), (1024, 3)])
def test_single_lane_equals_replay(kind, n, seed):
    import paper_2606_01693_amd as gq
    T = torch()
    q = make_queue(kind, n, lanes=64)
    rng = np.random.default_rng(seed)
    m = 3000
    ops = (rng.random(m) < 0.45).astype(np.uint8)  # 55% enqueues: reaches FULL often
    ops = 1 - ops
    args = np.arange(1, m + 1, dtype=np.uint64) * 7919
    h = gq.History(1, m)
    q.run_script(1, False, T.tensor(ops, device="cuda"),
                 T.tensor(args.view(np.int64), device="cuda"),
                 T.zeros(m, dtype=T.int16, device="cuda"),
                 T.tensor([m], dtype=T.int32, device="cuda"), m, h)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    proc, op, st, val, call, ret, _ = h.to_numpy()
    exp_st, exp_val, resid = oracle.fifo_replay(ops, args, capacity=cap_of(kind, n))
    assert np.array_equal(st, exp_st)
    assert np.array_equal(val, exp_val)
    assert np.array_equal(drain_fifo(q, n + 8 if BOUNDED[kind] else m), resid)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("seed", range(6))
def test_single_wave_closed_form(kind, seed):
    """Lemma 1: one wavefront's active lanes take consecutive tickets in lane
    order, so into a quiescent queue the r-th active enqueuer's item is the
    r-th dequeued, and the r-th active dequeuer receives it."""
    import paper_2606_01693_amd as gq
    T = torch()
    q = make_queue(kind, 256)
    rng = np.random.default_rng(100 + seed)
    enq_mask = rng.random(64) < rng.uniform(0.1, 1.0)
    enq_mask[rng.integers(0, 64)] = True
    deq_mask = rng.random(64) < rng.uniform(0.1, 1.0)
    deq_mask[rng.integers(0, 64)] = True
    args = (np.arange(64, dtype=np.uint64) + 1) * 1000003

    def run(mask, op):
        n_ops = T.tensor(mask.astype(np.int32), device="cuda")
        h = gq.History(64, 1)
        q.run_script(64, False, T.full((64,), op, dtype=T.uint8, device="cuda"),
                     T.tensor(args.view(np.int64), device="cuda"),
                     T.zeros(64, dtype=T.int16, device="cuda"), n_ops, 1, h)
        T.cuda.synchronize()
        return h.to_numpy()

    proc, op, st, val, _, _, _ = run(enq_mask, 0)
    assert (st == gq.GQ_OK).all() and np.array_equal(proc, np.nonzero(enq_mask)[0])
    proc, op, st, val, _, _, _ = run(deq_mask, 1)
    enq_lanes = np.nonzero(enq_mask)[0]
    deq_lanes = np.nonzero(deq_mask)[0]
    assert np.array_equal(proc, deq_lanes)
    for r, lane in enumerate(deq_lanes):
        if r < len(enq_lanes):
            assert st[r] == gq.GQ_OK and val[r] == args[enq_lanes[r]], (r, lane)
        else:
            assert st[r] == gq.GQ_EMPTY
    rest = drain_fifo(q, 64)
    assert np.array_equal(rest, args[enq_lanes[len(deq_lanes):]])


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("tg", [64, 0])
def test_batches_are_stream_ordered(kind, tg):
    import paper_2606_01693_amd as gq
    T = torch()
    n = 1 << 12
    q = make_queue(kind, n, ticket_group=tg)
    a = T.arange(1, 1001, dtype=T.int64, device="cuda")
    b = T.arange(5001, 6501, dtype=T.int64, device="cuda")
    nok = T.zeros(1, dtype=T.int64, device="cuda")
    q.enqueue_batch(a, num_ok=nok)
    q.enqueue_batch(b, num_ok=nok)
    out1 = T.zeros(1000, dtype=T.int64, device="cuda")
    out2 = T.zeros(1501, dtype=T.int64, device="cuda")
    st2 = T.zeros(1501, dtype=T.uint8, device="cuda")
    q.dequeue_batch(out1, num_ok=nok)
    q.dequeue_batch(out2, st2, num_ok=nok)
    T.cuda.synchronize()
    assert int(nok) == 2500 + 2500
    assert sorted(out1.cpu().tolist()) == list(range(1, 1001))
    s2 = st2.cpu().numpy()
    assert (s2 == gq.GQ_OK).sum() == 1500 and (s2 == gq.GQ_EMPTY).sum() == 1
    assert sorted(out2.cpu().numpy()[s2 == gq.GQ_OK].tolist()) == list(range(5001, 6501))
    assert q.check_error() == gq.GQ_OK


@pytest.mark.parametrize("kind", [k for k in KINDS if BOUNDED[k]])
@pytest.mark.parametrize("n", [2, 64, 1 << 14])
@pytest.mark.parametrize("tg", [64, 0])
def test_batch_capacity_exact(kind, n, tg):
    """With only enqueues in flight, a linearizable bounded queue accepts
    exactly capacity - size of them; with only dequeues, it returns exactly
    size items."""
    import paper_2606_01693_amd as gq
    T = torch()
    q = make_queue(kind, n, lanes=512, ticket_group=tg)
    m = n + 100
    items = T.arange(1, m + 1, dtype=T.int64, device="cuda")
    st = T.zeros(m, dtype=T.uint8, device="cuda")
    q.enqueue_batch(items, st)
    out = T.zeros(n + 50, dtype=T.int64, device="cuda")
    st2 = T.zeros(n + 50, dtype=T.uint8, device="cuda")
    q.dequeue_batch(out, st2)
    T.cuda.synchronize()
    s = st.cpu().numpy()
    assert (s == gq.GQ_OK).sum() == n and (s == gq.GQ_FULL).sum() == 100
    s2 = st2.cpu().numpy()
    assert (s2 == gq.GQ_OK).sum() == n and (s2 == gq.GQ_EMPTY).sum() == 50
    accepted = items.cpu().numpy()[s == gq.GQ_OK]
    assert sorted(out.cpu().numpy()[s2 == gq.GQ_OK].tolist()) == sorted(accepted.tolist())


# ---------------------------------------------------------------------------
# Small producer/consumer configuration: capacity 2^10, uint32 payload
# (pid << 20) | seq, 8 producer + 8 consumer wavefronts, 2^16 operations.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("run", range(5))
def test_c1_role_split(kind, run):
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(1, run)
    n, lanes, block = 1 << 10, 1024, 256
    # G-WFQ-YMC: every poll of an empty queue takes a cell; size its pool for
    # the consumers' polling
    q = make_queue(kind, n, width=4, lanes=lanes,
                   **({"ymc_pool_cells": 1 << 24} if kind == "ymc" else {}))
    prod_waves = workloads.producer_waves(seed, 16, 8)
    role = np.repeat(np.where(prod_waves, 0, 1), 64).astype(np.uint8)
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    h = gq.History(lanes, 1 << 15)  # every poll is recorded
    q.run_prodcons(seed, lanes, block, T.tensor(role, device="cuda"), 64, 32768, 0, 1, counts, h,
                   max_rounds=1 << 22)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] == 32768 and c[1] == 32768
    hist, overflow = history(h)
    assert overflow == 0
    drain = drain_fifo(q, n)
    rep = check_history(hist, drain, capacity=cap_of(kind, n), token_shift=20)
    assert_clean(rep, hist, drain, tag=f"c1split_{kind}_{run}")


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("run", range(5))
def test_c1_balanced(kind, run):
    """Every lane enqueues then dequeues, 32 times; 1024 lanes on capacity 1024:
    no FULL can occur, and no dequeue can find the queue empty (each dequeuer
    completed its own enqueue first)."""
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes = 1 << 10, 1024
    q = make_queue(kind, n, width=8, lanes=lanes)
    counts = T.zeros(4, dtype=T.int64, device="cuda")
    h = gq.History(lanes, 64)
    q.run_balanced(lanes, 32, counts, h)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    assert counts.cpu().tolist() == [32768, 32768, 0, 0]
    hist, overflow = history(h)
    assert overflow == 0
    drain = drain_fifo(q, n)
    rep = check_history(hist, drain, capacity=n)
    assert_clean(rep, hist, drain, tag=f"c1bal_{kind}_{run}")


# ---------------------------------------------------------------------------
# Tiny concurrent runs: exhaustive linearizability search
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("chunk", range(4))
def test_tiny_histories_linearizable(kind, chunk):
    import paper_2606_01693_amd as gq
    T = torch()
    rng = random.Random(4242 + chunk)
    n = 4
    q = make_queue(kind, n, lanes=64)
    max_ops = 4
    for trial in range(50):
        q.reset()
        # prefill tokens come from a producer id no lane uses
        pre = [(0xFFFF << 32) | (i + 1) for i in range(rng.randint(0, 2))]
        prefill(q, pre)
        lanes = rng.randint(2, 6)
        ops = np.zeros((lanes, max_ops), dtype=np.uint8)
        args = np.zeros((lanes, max_ops), dtype=np.uint64)
        pauses = np.zeros((lanes, max_ops), dtype=np.int16)
        n_ops = np.array([rng.randint(2, max_ops) for _ in range(lanes)], dtype=np.int32)
        for g in range(lanes):
            for r in range(max_ops):
                ops[g, r] = rng.random() < 0.5
                args[g, r] = (g << 32) | (r + 1)
                pauses[g, r] = rng.randint(0, 40)
        h = gq.History(lanes, max_ops)
        q.run_script(lanes, True, T.tensor(ops.ravel(), device="cuda"),
                     T.tensor(args.ravel().view(np.int64), device="cuda"),
                     T.tensor(pauses.ravel(), device="cuda"),
                     T.tensor(n_ops, device="cuda"), max_ops, h)
        T.cuda.synchronize()
        hist, _ = history(h)
        drain = drain_fifo(q, n + 4 if BOUNDED[kind] else 64)
        rows = list(zip(hist.proc.tolist(), hist.op.tolist(), hist.st.tolist(),
                        hist.val.tolist(), hist.call.tolist(), hist.ret.tolist()))
        tmax = int(hist.ret.max()) + 10
        rows += [(99, 1, 0, int(v), tmax + 2 * k, tmax + 2 * k + 1) for k, v in enumerate(drain)]
        rows += [(99, 1, 1, 0, tmax + 2 * len(drain), tmax + 2 * len(drain) + 1)]
        ok, _ = oracle.check_linearizable(rows, capacity=n if BOUNDED[kind] else None,
                                          prefill=pre)
        if not ok:
            import os
            os.makedirs("gpurun_out", exist_ok=True)
            with open(f"gpurun_out/fail_tiny_{kind}_{chunk}_{trial}.txt", "w") as f:
                f.write(f"prefill {pre}\n")
                for r in sorted(rows, key=lambda x: x[4]):
                    f.write(" ".join(str(x) for x in r) + "\n")
        assert ok, (trial, rows, pre)
        rep = check_history(hist, drain, prefill=pre, capacity=cap_of(kind, n))
        assert_clean(rep, hist, drain, pre, tag=f"tiny_{kind}_{chunk}_{trial}")
    assert q.check_error() == gq.GQ_OK


# ---------------------------------------------------------------------------
# Mixed 50/50 workload with recorded histories
# ---------------------------------------------------------------------------
def run_mix_checked(kind, n, lanes, ops, seed, slot_mode="linear", do_prefill=True, witness=None,
                    **opts):
    import paper_2606_01693_amd as gq
    T = torch()
    q = make_queue(kind, n, lanes=lanes, slot_mode=slot_mode, **opts)
    pre = []
    if do_prefill:
        pre = [int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)]
        prefill(q, pre)
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    h = gq.History(lanes, ops)
    q.run_mix(seed, lanes, ops, counts, h)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    hist, overflow = history(h)
    assert overflow == 0
    # the device drew the same roles as the shared workload definition
    roles = workloads.mix_roles(seed, lanes, ops).ravel()
    assert np.array_equal(hist.op, roles)
    c = counts.cpu().numpy().view(np.uint64).tolist()
    assert c[0] == int(((hist.op == 0) & (hist.st == 0)).sum())
    # the kernel's multiset checksums equal the oracle's over the recorded items
    assert (c[1], c[4], c[5]) == oracle.multiset_checksums(hist.deq_ok())
    assert (c[0], c[6], c[7]) == oracle.multiset_checksums(hist.enq_ok())
    expect = len(pre) + c[0] - c[1]
    drain = drain_fifo(q, n if BOUNDED[kind] else expect + 1)
    assert len(drain) == expect
    rep = check_history(hist, drain, prefill=pre, capacity=cap_of(kind, n), witness=witness)
    assert_clean(rep, hist, drain, pre,
                 tag=f"mix_{kind}_{n}_{lanes}_{ops}_{slot_mode}_tg{opts.get('ticket_group', 0)}")
    return c


# ticket_group 64: every wavefront takes its own tickets (WaveFAA alone);
# 0: the default workgroup aggregation (1024 lanes, or the largest power of
# two dividing the lane count).
TICKET_GROUPS = [64, 0]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n,lanes,ops", [(2, 512, 64), (4, 1536, 32), (64, 16384, 16),
                                         (1 << 10, 16384, 32), (1 << 16, 65536, 16)])
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_mix_history(kind, n, lanes, ops, tg):
    run_mix_checked(kind, n, lanes, ops, workloads.run_seed(2, n), ticket_group=tg)


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
@pytest.mark.parametrize("slot_mode", ["remap", "padded", "linear"])
@pytest.mark.parametrize("n", [4, 1 << 10])
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_mix_history_slot_layouts(kind, slot_mode, n, tg):
    """Every slot layout of the ring queues (remapped lines, padded, linear)
    under both ticket modes passes O3/O4/O6 on the whole history."""
    lanes = 1024 if n < 64 else 16384
    run_mix_checked(kind, n, lanes, 32, workloads.run_seed(2, 77), slot_mode=slot_mode,
                    ticket_group=tg)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [4, 1 << 10, 1 << 16])
def test_mix_history_fenced_handoff(kind, n):
    """The release/acquire payload hand-off (GQ_OPT_FENCED) passes the same checks."""
    lanes = 1024 if n < 64 else 16384  # G-WFQ's cycle bound at tiny capacity
    run_mix_checked(kind, n, lanes, 32, workloads.run_seed(2, 78), fenced=True)


def checksum_add(a, b):
    """Checksums (count, S1, S2) of the union of two multisets."""
    m = (1 << 64) - 1
    return a[0] + b[0], (a[1] + b[1]) & m, (a[2] + b[2]) & m


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_mix_timed_kernel_conserves(kind, tg):
    """The kernel the benchmark times, in the benchmark's own launch: no
    history, atomic hand-off, capacity 2^20, 2^26 attempts by the lanes the
    benchmark's step uses (the most lanes, up to 2^19, resident at once),
    prefill n/2.  O3 conservation at full size: the tokens the lanes enqueued
    (from their per-lane enqueue counts) and the prefill must equal, as a
    multiset, what the lanes dequeued plus what a sequential drain finds left
    (checksums: count and wrapping sums of v and v*v); the kernel's own
    enqueue checksums must equal the oracle's over those tokens; the drained
    residual must consist of distinct generated tokens, each producer's in
    increasing order (a FIFO's remainder)."""
    import paper_2606_01693_amd as gq
    T = torch()
    import bench
    n = 1 << 20
    lanes, ops = bench.step_shape(gq, kind, tg)
    assert lanes * ops == 1 << 26
    seed = workloads.run_seed(2, 1)
    q = make_queue(kind, n, lanes=lanes, ticket_group=tg,
                   **({"ymc_pool_cells": 1 << 27} if kind == "ymc" else {}))
    pre = np.array([int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)], dtype=np.uint64)
    q.enqueue_batch(T.tensor(pre.view(np.int64), device="cuda"))
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    lane_enq = T.zeros(lanes, dtype=T.int32, device="cuda")
    q.run_mix(seed, lanes, ops, counts, lane_enq=lane_enq)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    assert q.stats().dropped == 0
    c = counts.cpu().numpy().view(np.uint64).tolist()
    enq = oracle.mix_tokens_from_counts(lane_enq.cpu().numpy())
    assert oracle.multiset_checksums(enq) == (c[0], c[6], c[7])
    assert c[0] + c[1] + c[2] + c[3] == lanes * ops
    drain = drain_fifo(q, n if BOUNDED[kind] else len(pre) + c[0] - c[1] + 1)
    assert len(drain) == len(pre) + c[0] - c[1]
    put = checksum_add(oracle.multiset_checksums(pre), oracle.multiset_checksums(enq))
    out = checksum_add((c[1], c[4], c[5]), oracle.multiset_checksums(drain))
    assert put == out, (put, out)
    assert len(np.unique(drain)) == len(drain)
    rep = oracle.conservation(np.concatenate([pre, enq]), drain)
    assert rep["extra"] == 0, rep
    dh = oracle.History(np.zeros(len(drain)), np.ones(len(drain)), np.zeros(len(drain)), drain,
                        2 * np.arange(len(drain)), 2 * np.arange(len(drain)) + 1)
    assert oracle.producer_order(dh)["consumer_order"] == 0


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
@pytest.mark.parametrize("slot_mode", ["remap", "padded", "linear"])
def test_mix_group_kernel_conserves_every_layout(kind, slot_mode):
    """The group kernel without a history has a copy specialised for linear
    slots; both copies conserve the items on every slot layout: capacity
    2^16 prefilled to n/2, 2^14 lanes x 64 ops in 1024-lane workgroups, the
    prefill plus the enqueued tokens equal (checksums) the dequeued items
    plus the drain, and the kernel's enqueue checksums equal the oracle's
    over the tokens its per-lane counts name."""
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes, ops = 1 << 16, 1 << 14, 64
    q = make_queue(kind, n, lanes=lanes, slot_mode=slot_mode, ticket_group=1024)
    pre = np.array([int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)], dtype=np.uint64)
    q.enqueue_batch(T.tensor(pre.view(np.int64), device="cuda"))
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    lane_enq = T.zeros(lanes, dtype=T.int32, device="cuda")
    q.run_mix(workloads.run_seed(2, 7), lanes, ops, counts, lane_enq=lane_enq)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().numpy().view(np.uint64).tolist()
    enq = oracle.mix_tokens_from_counts(lane_enq.cpu().numpy())
    assert oracle.multiset_checksums(enq) == (c[0], c[6], c[7])
    assert c[0] + c[1] + c[2] + c[3] == lanes * ops
    drain = drain_fifo(q, n)
    put = checksum_add(oracle.multiset_checksums(pre), oracle.multiset_checksums(enq))
    out = checksum_add((c[1], c[4], c[5]), oracle.multiset_checksums(drain))
    assert put == out, (put, out)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_mix_full_size(kind, tg):
    """The benchmark's configuration: capacity 2^20, 2048 x 256 lanes, 2^26
    operations, prefill n/2; the full history is checked, and in the
    benchmark's own launch (default ticket group) a linearization of all
    2^26 operations plus the drain is found and confirmed (O10)."""
    run_mix_checked(kind, 1 << 20, 2048 * 256, 128, workloads.run_seed(2, 0), ticket_group=tg,
                    witness=(tg == 0))


# ---------------------------------------------------------------------------
# G-WFQ slow path, forced: patience 0 sends every operation through the
# request/helping path; help delay 1 makes every lane inspect a peer record
# on every operation.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,lanes,ops,patience,delay", [
    (4, 256, 16, 0, 1), (64, 1024, 16, 0, 1), (64, 1024, 16, 1, 1), (1 << 10, 4096, 16, 0, 4),
    (1 << 10, 4096, 16, 2, 64), (16, 2048, 16, 0, 1),
])
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_wfq_forced_slow_path_mix(n, lanes, ops, patience, delay, tg):
    run_mix_checked("wfq", n, lanes, ops, workloads.run_seed(3, n + patience),
                    patience=patience, help_delay=delay, ticket_group=tg)


@pytest.mark.parametrize("run", range(3))
def test_wfq_forced_slow_path_role_split(run):
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(1, 100 + run)
    n, lanes, block = 1 << 10, 1024, 256
    q = make_queue("wfq", n, width=4, lanes=lanes, patience=0, help_delay=1)
    prod_waves = workloads.producer_waves(seed, 16, 8)
    role = np.repeat(np.where(prod_waves, 0, 1), 64).astype(np.uint8)
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    h = gq.History(lanes, 1 << 14)
    q.run_prodcons(seed, lanes, block, T.tensor(role, device="cuda"), 16, 8192, 0, 1, counts, h,
                   max_rounds=1 << 22)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] == 8192 and c[1] == 8192
    hist, overflow = history(h)
    assert overflow == 0
    drain = drain_fifo(q, n)
    rep = check_history(hist, drain, capacity=n, token_shift=20)
    assert_clean(rep, hist, drain, tag=f"wfq_slow_split_{run}")
    st = q.stats()
    assert st.slow_enter > 0


@pytest.mark.parametrize("chunk", range(2))
def test_wfq_tiny_histories_slow_path(chunk):
    """Exhaustive linearizability on tiny runs with every op on the slow path."""
    import paper_2606_01693_amd as gq
    T = torch()
    rng = random.Random(777 + chunk)
    n = 4
    q = make_queue("wfq", n, lanes=64, patience=0, help_delay=1)
    max_ops = 4
    for trial in range(50):
        q.reset()
        pre = [(0xFFFF << 32) | (i + 1) for i in range(rng.randint(0, 2))]
        prefill(q, pre)
        lanes = rng.randint(2, 6)
        ops = np.zeros((lanes, max_ops), dtype=np.uint8)
        args = np.zeros((lanes, max_ops), dtype=np.uint64)
        pauses = np.zeros((lanes, max_ops), dtype=np.int16)
        n_ops = np.array([rng.randint(2, max_ops) for _ in range(lanes)], dtype=np.int32)
        for g in range(lanes):
            for r in range(max_ops):
                ops[g, r] = rng.random() < 0.5
                args[g, r] = (g << 32) | (r + 1)
                pauses[g, r] = rng.randint(0, 40)
        h = gq.History(lanes, max_ops)
        q.run_script(lanes, True, T.tensor(ops.ravel(), device="cuda"),
                     T.tensor(args.ravel().view(np.int64), device="cuda"),
                     T.tensor(pauses.ravel(), device="cuda"),
                     T.tensor(n_ops, device="cuda"), max_ops, h)
        T.cuda.synchronize()
        hist, _ = history(h)
        drain = drain_fifo(q, n + 4)
        rows = list(zip(hist.proc.tolist(), hist.op.tolist(), hist.st.tolist(),
                        hist.val.tolist(), hist.call.tolist(), hist.ret.tolist()))
        tmax = int(hist.ret.max()) + 10
        rows += [(99, 1, 0, int(v), tmax + 2 * k, tmax + 2 * k + 1) for k, v in enumerate(drain)]
        rows += [(99, 1, 1, 0, tmax + 2 * len(drain), tmax + 2 * len(drain) + 1)]
        ok, _ = oracle.check_linearizable(rows, capacity=n, prefill=pre)
        assert ok, (trial, rows, pre)
        rep = check_history(hist, drain, prefill=pre, capacity=n)
        assert_clean(rep, hist, drain, pre, tag=f"wfq_tiny_slow_{chunk}_{trial}")
    assert q.check_error() == gq.GQ_OK


# ---------------------------------------------------------------------------
# G-WFQ-YMC slow path, forced (patience 0), and the pool-exhaustion latch.
# ---------------------------------------------------------------------------
# (the 16384-lane case races slow-path enqueue claims against dequeuers
# marking the same cells, where a helper must commit a claim it lost to the
# owner for its own cell)
@pytest.mark.parametrize("n,lanes,ops,patience", [(64, 1024, 16, 0), (1 << 10, 4096, 16, 1),
                                                   (16, 2048, 16, 0), (1 << 10, 16384, 32, 1)])
@pytest.mark.parametrize("tg", TICKET_GROUPS)
def test_ymc_forced_slow_path_mix(n, lanes, ops, patience, tg):
    run_mix_checked("ymc", n, lanes, ops, workloads.run_seed(4, n + patience), patience=patience,
                    ticket_group=tg)


@pytest.mark.parametrize("run", range(2))
def test_ymc_forced_slow_path_role_split(run):
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(1, 200 + run)
    n, lanes, block = 1 << 10, 1024, 256
    # consumers poll an often-empty queue and every poll takes a cell: size
    # the pool for the polling, not for the 8192 items
    q = make_queue("ymc", n, width=4, lanes=lanes, patience=0, ymc_pool_cells=1 << 24)
    prod_waves = workloads.producer_waves(seed, 16, 8)
    role = np.repeat(np.where(prod_waves, 0, 1), 64).astype(np.uint8)
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    h = gq.History(lanes, 1 << 14)
    q.run_prodcons(seed, lanes, block, T.tensor(role, device="cuda"), 16, 8192, 0, 1, counts, h,
                   max_rounds=1 << 22)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] == 8192 and c[1] == 8192
    hist, overflow = history(h)
    assert overflow == 0
    drain = drain_fifo(q, 64)
    rep = check_history(hist, drain, capacity=0, token_shift=20)
    assert_clean(rep, hist, drain, tag=f"ymc_slow_split_{run}")


@pytest.mark.parametrize("patience", [0, 2])
def test_ymc_slow_enqueue_after_empty_burst(patience):
    """Dequeuers that found the queue empty leave their cells unusable; the
    enqueues that follow land on those cells, fail their fast attempts and
    complete on the slow path.  Every item must still come out, in batches'
    order."""
    import paper_2606_01693_amd as gq
    T = torch()
    q = make_queue("ymc", 1 << 10, lanes=4096, patience=patience)
    out = T.zeros(4096, dtype=T.int64, device="cuda")
    st = T.zeros(4096, dtype=T.uint8, device="cuda")
    q.dequeue_batch(out, st)              # 4096 EMPTY: H runs ahead of T
    items = T.arange(1, 3001, dtype=T.int64, device="cuda")
    st_e = T.zeros(3000, dtype=T.uint8, device="cuda")
    q.enqueue_batch(items, st_e)
    out2 = T.zeros(3000, dtype=T.int64, device="cuda")
    st2 = T.zeros(3000, dtype=T.uint8, device="cuda")
    q.dequeue_batch(out2, st2)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    assert (st.cpu().numpy() == gq.GQ_EMPTY).all()
    assert (st_e.cpu().numpy() == gq.GQ_OK).all()
    assert (st2.cpu().numpy() == gq.GQ_OK).all()
    assert sorted(out2.cpu().tolist()) == list(range(1, 3001))
    assert q.stats().slow_enter > 0


def test_ymc_pool_exhaustion_latches():
    """Running past the preallocated pool reports GQ_ERR_POOL_EXHAUSTED."""
    import paper_2606_01693_amd as gq
    T = torch()
    q = gq.Queue("ymc", 64, item_width=8, max_threads=256, ymc_pool_cells=512)
    items = T.arange(1, 1001, dtype=T.int64, device="cuda")
    st = T.zeros(1000, dtype=T.uint8, device="cuda")
    q.enqueue_batch(items, st)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_ERR_POOL_EXHAUSTED
    s = st.cpu().numpy().astype(np.int8)
    assert (s == gq.GQ_OK).sum() <= 512
