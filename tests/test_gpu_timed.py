"""Fixed-duration runs (the paper's balanced and split micro-benchmark
kernels, Section V-A): the windowed counts are plausible; recorded runs pass
the oracle's history checks (O3/O4/O6 and a linearization witness, O10); at
the benchmark's size the whole run is conserved (multiset checksums of what
went in and out, with the drain); and what is left in the queue afterwards is
a valid FIFO remainder -- distinct tokens, each from the prefill or from a
lane of the run, every producer's tokens in the order it enqueued them -- of
a size the bounded queue can hold."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_clean, check_history, drain_fifo, history, prefill, torch

pytestmark = pytest.mark.gpu


def check_remainder(drain, lanes, cap):
    toks = np.asarray(drain, dtype=np.uint64)
    assert len(np.unique(toks)) == len(toks), "duplicate tokens in the remainder"
    if cap:
        assert len(toks) <= cap
    prod = (toks >> np.uint64(32)).astype(np.int64)
    seq = (toks & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert ((prod < lanes) | (prod == 0xFFFFFFFF)).all(), "token from no producer of the run"
    assert (seq >= 1).all()
    for p in np.unique(prod):
        s = seq[prod == p]
        assert (np.diff(s) > 0).all(), f"producer {p}: remainder out of enqueue order"


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_timed_balanced(kind):
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes = 1 << 14, 4096
    print(f"[case] timed balanced kind={kind} n={n} lanes={lanes}", flush=True)
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes,
                 ymc_pool_cells=(1 << 26) if kind == "ymc" else 0)
    pre = T.tensor(np.array([int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)],
                            dtype=np.uint64).view(np.int64), device="cuda")
    q.enqueue_batch(pre)
    counts = T.zeros(10, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    q.run_timed("balanced", lanes, counts, ctl, warmup_us=200, window_us=2000)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] > 0 and c[1] > 0 and c[2] == 0 and c[3] == 0, c
    assert abs(c[0] - c[1]) <= lanes, c  # each lane alternates enqueue and dequeue
    check_remainder(drain_fifo(q, n + 1 if kind != "ymc" else 2 * n), lanes,
                    n if kind != "ymc" else 0)


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
def test_timed_producers_only_fill_exactly(kind):
    """Every wavefront a producer: a bounded queue ends exactly full."""
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes = 1 << 12, 2048
    print(f"[case] timed producers-only kind={kind}", flush=True)
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes)
    counts = T.zeros(10, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    q.run_timed("split", lanes, counts, ctl, prod_pct=100, warmup_us=0, window_us=1000)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[2] > 0 and c[1] == 0 and c[3] == 0, c
    drain = drain_fifo(q, n + 1)
    assert len(drain) == n
    check_remainder(drain, lanes, n)


def test_timed_split_half(kind="lfq"):
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes = 1 << 14, 8192
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes)
    counts = T.zeros(10, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    q.run_timed("split", lanes, counts, ctl, prod_pct=50, warmup_us=200, window_us=2000)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] > 0 and c[1] > 0, c
    check_remainder(drain_fifo(q, n + 1), lanes, n)


def checksum_add(a, b):
    m = (1 << 64) - 1
    return a[0] + b[0], (a[1] + b[1]) & m, (a[2] + b[2]) & m


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
@pytest.mark.parametrize("mode,pct", [("balanced", 50), ("split", 25), ("split", 75)])
def test_timed_history_oracle(kind, mode, pct):
    """4096 lanes, capacity 2^12 prefilled to n/2, 1.2 ms: every operation of
    the run recorded (a lane stops when its 2048-entry row is full) and the
    whole history checked with the sequential drain appended."""
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes, per_lane = 1 << 12, 4096, 2048
    print(f"[case] timed history kind={kind} mode={mode} pct={pct}", flush=True)
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes,
                 ymc_pool_cells=(1 << 26) if kind == "ymc" else 0)
    pre = [int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)]
    prefill(q, pre)  # in list order: the oracle takes it as the initial queue
    counts = T.zeros(10, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    h = gq.History(lanes, per_lane)
    q.run_timed(mode, lanes, counts, ctl, prod_pct=pct, warmup_us=200, window_us=1000, hist=h)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().numpy().view(np.uint64).tolist()
    hist, overflow = history(h)
    assert overflow == 0
    assert c[8] == int(((hist.op == 0) & (hist.st == 0)).sum())
    assert (c[9], c[4], c[5]) == oracle.multiset_checksums(hist.deq_ok())
    assert (c[8], c[6], c[7]) == oracle.multiset_checksums(hist.enq_ok())
    expect = len(pre) + c[8] - c[9]
    drain = drain_fifo(q, n if kind != "ymc" else expect + 1)
    assert len(drain) == expect
    rep = check_history(hist, drain, prefill=pre, capacity=n if kind != "ymc" else 0)
    assert_clean(rep, hist, drain, pre, tag=f"timed_{kind}_{mode}{pct}")


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_timed_full_size_conservation(kind):
    """The benchmark's largest fixed-duration run, balanced: 32768 lanes,
    capacity 2^20 prefilled to n/2, 1 ms + 5 ms.  The prefill and the tokens
    the lanes enqueued (from their per-lane counts) equal, as multisets, what
    the lanes dequeued plus the drain (count and wrapping sums of v, v*v)."""
    import paper_2606_01693_amd as gq
    T = torch()
    n, lanes = 1 << 20, 32768
    print(f"[case] timed full size kind={kind}", flush=True)
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes,
                 ymc_pool_cells=(1 << 28) if kind == "ymc" else 0)
    pre = np.array([int(workloads.token(0xFFFFFFFF, i)) for i in range(n // 2)], dtype=np.uint64)
    q.enqueue_batch(T.tensor(pre.view(np.int64), device="cuda"))
    counts = T.zeros(10, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    lane_enq = T.zeros(lanes, dtype=T.int32, device="cuda")
    q.run_timed("balanced", lanes, counts, ctl, warmup_us=1000, window_us=5000,
                lane_enq=lane_enq)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().numpy().view(np.uint64).tolist()
    enq = oracle.mix_tokens_from_counts(lane_enq.cpu().numpy())
    assert oracle.multiset_checksums(enq) == (c[8], c[6], c[7])
    drain = drain_fifo(q, n if kind != "ymc" else len(pre) + c[8] - c[9] + 1)
    assert len(drain) == len(pre) + c[8] - c[9]
    put = checksum_add(oracle.multiset_checksums(pre), oracle.multiset_checksums(enq))
    out = checksum_add((c[9], c[4], c[5]), oracle.multiset_checksums(drain))
    assert put == out, (put, out)
    check_remainder(drain, lanes, n if kind != "ymc" else 0)
