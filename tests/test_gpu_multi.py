"""Many independent queues in one launch (and captured in a hipGraph): every
queue's recorded history passes the oracle's checks on its own, and graph
replays keep each queue's books balanced."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_clean, check_history, drain_fifo, torch
import oracle

pytestmark = pytest.mark.gpu


def build(kind, caps, **opts):
    """One wavefront per 64 slots of capacity (at least one)."""
    import paper_2606_01693_amd as gq
    lanes = [64 * max(1, c // 64) for c in caps]
    qs = [gq.Queue(kind, c, item_width=8, max_threads=l, **opts) for c, l in zip(caps, lanes)]
    return qs, lanes


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_multi_queue_histories(kind):
    import paper_2606_01693_amd as gq
    T = torch()
    rng = np.random.default_rng(5)
    caps = [int(2 ** e) for e in rng.integers(4, 11, size=24)]
    qs, lanes = build(kind, caps)
    if sum(lanes) % 256:
        lanes[-1] += 256 - sum(lanes) % 256
        qs[-1] = gq.Queue(kind, caps[-1], item_width=8, max_threads=lanes[-1])
    print(f"[case] kind={kind} caps={caps} lanes={lanes}", flush=True)
    m = gq.Multi(qs, lanes, block=256)
    ops = 16
    counts = T.zeros(8 * len(qs), dtype=T.int64, device="cuda")
    total = sum(lanes)
    h = gq.History(total, ops)
    seed = workloads.run_seed(5, 0)
    m.run_mix(seed, ops, counts, h)
    T.cuda.synchronize()
    proc, op, st, val, call, ret, overflow = h.to_numpy()
    assert overflow == 0
    # the device drew each lane's roles from the shared workload definition
    assert np.array_equal(op, workloads.mix_roles(seed, total, ops).ravel())
    c = counts.cpu().numpy().reshape(-1, 8)
    lane0 = np.concatenate([[0], np.cumsum(lanes)])
    for i, q in enumerate(qs):
        assert q.check_error() == gq.GQ_OK, i
        sel = (proc >= lane0[i]) & (proc < lane0[i + 1])
        hist = oracle.History(proc[sel], op[sel], st[sel], val[sel], call[sel], ret[sel])
        assert c[i, 0] == int(((hist.op == 0) & (hist.st == 0)).sum())
        expect = int(c[i, 0] - c[i, 1])
        drain = drain_fifo(q, caps[i] if kind != "ymc" else expect + 1)
        assert len(drain) == expect
        rep = check_history(hist, drain, capacity=caps[i] if kind != "ymc" else 0)
        assert_clean(rep, hist, drain, tag=f"multi_{kind}_{i}")
    m.close()


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
def test_multi_queue_graph_replays(kind):
    """Replay the captured launch several times with eager work in between;
    after every replay each queue's size equals enqueued minus dequeued."""
    import paper_2606_01693_amd as gq
    T = torch()
    caps = [256, 512, 1024, 2048, 256, 4096, 512, 256]
    lanes = [64 * max(1, c // 256) for c in caps]
    lanes[-1] += (256 - sum(lanes) % 256) % 256
    qs = [gq.Queue(kind, c, item_width=8, max_threads=l) for c, l in zip(caps, lanes)]
    m = gq.Multi(qs, lanes, block=256)
    s = T.cuda.Stream()
    counts = T.zeros(8 * len(qs), dtype=T.int64, device="cuda")
    with T.cuda.stream(s):
        m.capture(workloads.run_seed(5, 1), 8, counts, s)
    s.synchronize()
    size = np.zeros(len(qs), dtype=np.int64)
    prev = np.zeros((len(qs), 8), dtype=np.int64)
    for rep in range(4):
        with T.cuda.stream(s):
            m.replay(s)
        s.synchronize()
        c = counts.cpu().numpy().reshape(-1, 8)
        d = c - prev
        prev = c.copy()
        assert (d[:, 0] + d[:, 1] + d[:, 2] + d[:, 3] == np.array(lanes) * 8).all(), rep
        size += d[:, 0] - d[:, 1]
        assert ((size >= 0) & (size <= np.array(caps))).all()
        # eager work between replays: drain one queue completely and refill it
        qi = rep % len(qs)
        got = drain_fifo(qs[qi], caps[qi])
        assert len(got) == size[qi]
        size[qi] = 0
    for i, q in enumerate(qs):
        assert q.check_error() == gq.GQ_OK
        got = drain_fifo(q, caps[i])
        assert len(got) == size[i]
        # every token left belongs to one of this queue's lanes
        lane0 = sum(lanes[:i])
        prod = (np.asarray(got, dtype=np.uint64) >> np.uint64(32)).astype(np.int64)
        assert ((prod >= lane0) & (prod < lane0 + lanes[i])).all()
    m.close()


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_multi_queue_graph_replay_histories(kind):
    """The batched form at its configured shape -- 256 queues of capacity 2^e,
    e uniform in 8..16 (seeded), one wavefront per 256 slots, 16 operations
    per lane -- captured in a hipGraph with a history: after each of three
    replays, with eager drains in between, every queue's history of that
    replay passes O3/O4/O6 and yields a linearization witness (O10)."""
    import paper_2606_01693_amd as gq
    T = torch()
    rng = np.random.default_rng(workloads.run_seed(5, 0))
    caps = [int(2 ** e) for e in rng.integers(8, 17, size=256)]
    lanes = [64 * max(1, c // 256) for c in caps]
    lanes[int(np.argmax(caps))] += (-sum(lanes)) % 256
    qs = [gq.Queue(kind, c, item_width=8, max_threads=l,
                   **({"ymc_pool_cells": 16 * l * 16 + 4 * c} if kind == "ymc" else {}))
          for c, l in zip(caps, lanes)]
    print(f"[case] graph replay histories kind={kind} queues=256 lanes={sum(lanes)}", flush=True)
    m = gq.Multi(qs, lanes, block=256)
    ops = 16
    total = sum(lanes)
    counts = T.zeros(8 * len(qs), dtype=T.int64, device="cuda")
    h = gq.History(total, ops)
    s = T.cuda.Stream()
    seed = workloads.run_seed(5, 2)
    with T.cuda.stream(s):
        m.capture(seed, ops, counts, s, hist=h)
    s.synchronize()
    lane0 = np.concatenate([[0], np.cumsum(lanes)])
    prev = np.zeros((len(qs), 8), dtype=np.int64)
    for rep in range(3):
        with T.cuda.stream(s):
            m.replay(s)
        s.synchronize()
        c = counts.cpu().numpy().reshape(-1, 8)
        d = c - prev
        prev = c.copy()
        proc, op, st, val, call, ret, overflow = h.to_numpy()
        assert overflow == 0
        # replay r draws with seed + r + 1 (the captured seed bump)
        assert np.array_equal(op, workloads.mix_roles(seed + rep + 1, total, ops).ravel())
        for i, q in enumerate(qs):
            assert q.check_error() == gq.GQ_OK, i
            sel = (proc >= lane0[i]) & (proc < lane0[i + 1])
            hist = oracle.History(proc[sel], op[sel], st[sel], val[sel], call[sel], ret[sel])
            assert d[i, 0] == int(((hist.op == 0) & (hist.st == 0)).sum())
            expect = int(d[i, 0] - d[i, 1])
            drain = drain_fifo(q, caps[i] if kind != "ymc" else expect + 1)
            assert len(drain) == expect, (rep, i)
            rep_ = check_history(hist, drain, capacity=caps[i] if kind != "ymc" else 0)
            assert_clean(rep_, hist, drain, tag=f"graph_{kind}_{rep}_{i}")
    m.close()
