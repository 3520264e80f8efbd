"""Fixed-duration runs (the paper's balanced and split micro-benchmark
kernels, Section V-A): the windowed counts are plausible, and what is left in
the queue afterwards is a valid FIFO remainder -- distinct tokens, each from
the prefill or from a lane of the run, every producer's tokens in the order
it enqueued them -- of a size the bounded queue can hold."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import drain_fifo, torch

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
    counts = T.zeros(4, dtype=T.int64, device="cuda")
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
    counts = T.zeros(4, dtype=T.int64, device="cuda")
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
    counts = T.zeros(4, dtype=T.int64, device="cuda")
    ctl = T.zeros(4, dtype=T.int64, device="cuda")
    q.run_timed("split", lanes, counts, ctl, prod_pct=50, warmup_us=200, window_us=2000)
    T.cuda.synchronize()
    assert q.check_error() == gq.GQ_OK
    c = counts.cpu().tolist()
    assert c[0] > 0 and c[1] > 0, c
    check_remainder(drain_fifo(q, n + 1), lanes, n)
