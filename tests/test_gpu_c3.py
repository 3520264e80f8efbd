"""Imbalanced producer/consumer runs (the paper's split-kernel shape with
producer fractions away from 1/2, Section V-A): capacity 2^16, 1024
wavefronts of which the seed makes 128, 512 or 896 producers; in each round a
lane is active with probability 1, 1/2 or 1/64; producers retry on FULL and
consumers on EMPTY until every produced item was taken.

At full size the check is exact conservation through multiset checksums (the
wrapping sums of v and v*v of every item enqueued and dequeued, against the
same sums over the token set, enumerated here) plus an empty queue
afterwards.  A smaller run of the same shape records its whole history and
passes the oracle's conservation, per-producer order and violation checks."""
import time

import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_clean, check_history, drain_fifo, history, torch

pytestmark = pytest.mark.gpu

KINDS = ["lfq", "wfq", "ymc"]


def token_sums(role: np.ndarray, quota: int):
    """Wrapping sums of v and v*v over the tokens (g << 32) | (s + 1),
    s < quota, of every producer lane g."""
    g = np.nonzero(role == 0)[0].astype(np.uint64)
    s = np.arange(1, quota + 1, dtype=np.uint64)
    tok = ((g[:, None] << np.uint64(32)) | s[None, :]).ravel()
    with np.errstate(over="ignore"):
        return int(tok.sum(dtype=np.uint64)), int((tok * tok).sum(dtype=np.uint64))


def c3_run(kind, n, waves, prod_waves, log2_inv_p, items, seed, hist_per_lane=0,
           ymc_pool=1 << 30):
    import paper_2606_01693_amd as gq
    T = torch()
    lanes = waves * 64
    print(f"[case] c3 kind={kind} n={n} waves={waves} producers={prod_waves} "
          f"p=2^-{log2_inv_p} items={items} seed={seed}", flush=True)
    q = gq.Queue(kind, n, item_width=8, max_threads=lanes,
                 ymc_pool_cells=ymc_pool if kind == "ymc" else 0)
    mask = workloads.producer_waves(seed, waves, prod_waves)
    role = np.repeat(np.where(mask, 0, 1), 64).astype(np.uint8)
    plane = prod_waves * 64
    quota = -(-items // plane)
    target = quota * plane
    counts = T.zeros(8, dtype=T.int64, device="cuda")
    h = gq.History(lanes, hist_per_lane) if hist_per_lane else None
    # G-WFQ-YMC takes a cell for every poll of an empty queue: its pool (2^30
    # cells, 32 GiB) is sized for the consumers' polling, not for the items
    role_t = T.tensor(role, device="cuda")
    T.cuda.synchronize()
    t0 = time.perf_counter()
    q.run_prodcons(seed, lanes, 256, role_t, quota, target, log2_inv_p, 0, counts, h,
                   max_rounds=1 << 30, time_limit_ms=60000)
    T.cuda.synchronize()
    dt = time.perf_counter() - t0
    c = counts.cpu().numpy().view(np.uint64).tolist()
    st = q.stats()
    print(f"[c3] {dt:.2f} s counts(ok_enq, ok_deq, full, empty)={c[:4]} target={target} "
          f"cas_fail={st.cas_fail} slow={st.slow_enter}", flush=True)
    assert q.check_error() == gq.GQ_OK, gq.status_str(q.check_error())
    return q, role, quota, target, c, h


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prod_waves", [128, 512, 896])
@pytest.mark.parametrize("log2_inv_p", [0, 1, 6])
def test_c3_full_size_conservation(kind, prod_waves, log2_inv_p):
    T = torch()
    seed = workloads.run_seed(3, prod_waves + log2_inv_p)
    q, role, quota, target, c, _ = c3_run(kind, 1 << 16, 1024, prod_waves, log2_inv_p,
                                          1 << 23, seed)
    assert c[0] == target and c[1] == target
    s1, s2 = token_sums(role, quota)
    assert (c[6], c[7]) == (s1, s2), "enqueued tokens differ from the generated set"
    assert (c[4], c[5]) == (s1, s2), "dequeued multiset differs from the enqueued one"
    if kind != "ymc":
        assert len(drain_fifo(q, 64)) == 0
    else:
        out = T.zeros(4096, dtype=T.int64, device="cuda")
        st = T.zeros(4096, dtype=T.uint8, device="cuda")
        q.dequeue_batch(out, st)
        T.cuda.synchronize()
        assert int((st == 0).sum()) == 0


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prod_waves", [8, 56])
@pytest.mark.parametrize("log2_inv_p", [0, 6])
def test_c3_shape_histories(kind, prod_waves, log2_inv_p):
    """64 wavefronts, capacity 2^10, 2^15 items, whole history recorded."""
    seed = workloads.run_seed(3, 100 + prod_waves + log2_inv_p)
    n = 1 << 10
    q, role, quota, target, c, h = c3_run(kind, n, 64, prod_waves, log2_inv_p, 1 << 15, seed,
                                          hist_per_lane=1 << 14, ymc_pool=1 << 22)
    assert c[0] == target and c[1] == target
    hist, overflow = history(h)
    assert overflow == 0
    drain = drain_fifo(q, n)
    rep = check_history(hist, drain, capacity=n if kind != "ymc" else 0)
    assert_clean(rep, hist, drain, tag=f"c3_{kind}_{prod_waves}_{log2_inv_p}")
