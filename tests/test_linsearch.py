"""O10, the linearization witness search (Section IV, "Linearizability via
Porcupine"), pinned by the exhaustive search O5 (itself pinned by plain
permutation enumeration), by an independent witness check (O2 replay plus a
real-time check) and by legal-by-construction histories far too large for O5.
"""
import collections
import random

import numpy as np
import pytest

import oracle
from oracle import OP_DEQ, OP_ENQ, ST_EMPTY, ST_FULL, ST_OK
from oracle.linearize import check_linearizable
from test_oracle import CATALOGUE, legal_history


def hist(rows):
    return oracle.History.from_rows(rows)


def with_drain(rows, drain, final_empty=True):
    """The drain as O5 sees it: sequential dequeues after everything."""
    base = 10 ** 7
    out = list(rows) + [(99, OP_DEQ, ST_OK, v, base + 2 * k, base + 2 * k + 1)
                        for k, v in enumerate(drain)]
    if final_empty:
        out.append((99, OP_DEQ, ST_EMPTY, 0, base + 2 * len(drain), base + 2 * len(drain) + 1))
    return out


@pytest.mark.parametrize("rows,expected", CATALOGUE)
def test_catalogue(rows, expected):
    h = hist(rows)
    rc, order, _ = oracle.lin_witness(h, drain_ends_empty=False)
    assert rc == (1 if expected else 0)
    if rc == 1:
        assert oracle.check_witness(h, order, drain_ends_empty=False) == ""


def mutate(rng, rows, resid):
    """One plausible queue bug: two dequeue results swapped, an OK dequeue
    answered EMPTY (its item left for the drain), a timestamp moved, an EMPTY
    answer moved earlier, or the drain reordered."""
    rows = [list(r) for r in rows]
    kind = rng.randrange(6)
    deqs = [i for i, r in enumerate(rows) if r[1] == OP_DEQ and r[2] == ST_OK]
    if kind == 0 and len(deqs) >= 2:
        a, b = rng.sample(deqs, 2)
        rows[a][3], rows[b][3] = rows[b][3], rows[a][3]
    elif kind == 1 and deqs:
        i = rng.choice(deqs)
        rows[i][2] = ST_EMPTY
        resid = resid + [rows[i][3]]
        rows[i][3] = 0
    elif kind == 2:
        i = rng.randrange(len(rows))
        rows[i][4] = max(0, rows[i][4] + rng.randint(-30, 30))
        rows[i][5] = max(rows[i][4], rows[i][5] + rng.randint(-30, 30))
    elif kind == 3:
        e = [i for i, r in enumerate(rows) if r[1] == OP_DEQ and r[2] == ST_EMPTY]
        if e:
            i = rng.choice(e)
            rows[i][4] = max(0, rows[i][4] - 40)
    elif kind == 4 and len(resid) >= 2:
        resid = list(resid)
        i, j = rng.sample(range(len(resid)), 2)
        resid[i], resid[j] = resid[j], resid[i]
    return [tuple(r) for r in rows], resid


@pytest.mark.parametrize("chunk", range(8))
def test_agrees_with_bruteforce(chunk):
    """On tiny histories (legal ones and mutated ones, bounded and unbounded,
    with prefill and drain) the exhaustive mode answers exactly as O5, every
    witness passes the independent check, and the greedy mode (one candidate
    per branch) never contradicts O5."""
    seen = collections.Counter()
    for seed in range(chunk * 250, (chunk + 1) * 250):
        rng = random.Random(seed)
        cap = rng.choice([None, 2, 3])
        pre = list(range(1, rng.randint(0, 2) + 1))
        rows, resid = legal_history(rng, rng.randint(1, 9), rng.randint(1, 4), capacity=cap,
                                    prefill=pre)
        if rng.random() < 0.7:
            rows, resid = mutate(rng, rows, resid)
        lin = check_linearizable(with_drain(rows, resid), capacity=cap, prefill=pre)[0]
        h = hist(rows)
        rc, order, _ = oracle.lin_witness(h, prefill=pre, drain=resid, capacity=cap or 0)
        assert rc == (1 if lin else 0), (seed, rows, resid, pre, cap)
        if rc == 1:
            assert oracle.check_witness(h, order, prefill=pre, drain=resid,
                                        capacity=cap or 0) == ""
        g, _, _ = oracle.lin_witness(h, prefill=pre, drain=resid, capacity=cap or 0, width=1,
                                     budget=10 ** 5)
        assert g in ((1, -1) if lin else (0, -1)), seed
        seen[(lin, g)] += 1
    # the greedy mode decides the legal ones without backtracking into a miss
    assert seen[(True, -1)] == 0


def test_drain_without_final_empty_and_item_left_over():
    """An item never dequeued nor drained: with the drain's final EMPTY the
    history is not linearizable (the item was lost), without it it is."""
    rows = [(0, OP_ENQ, ST_OK, 5, 0, 1), (0, OP_ENQ, ST_OK, 6, 2, 3),
            (1, OP_DEQ, ST_OK, 5, 4, 5)]
    assert oracle.lin_witness(hist(rows), drain=[], drain_ends_empty=True)[0] == 0
    assert oracle.lin_witness(hist(rows), drain=[], drain_ends_empty=False)[0] == 1
    assert oracle.lin_witness(hist(rows), drain=[6], drain_ends_empty=True)[0] == 1


def test_capacity_bound():
    """Two overlapping OK enqueues into a queue of capacity 1 holding a
    prefilled item, no dequeue in between: illegal at capacity 1 and 2,
    legal at 3 and unbounded."""
    rows = [(0, OP_ENQ, ST_OK, 5, 0, 10), (1, OP_ENQ, ST_OK, 6, 0, 10)]
    for cap, want in ((1, 0), (2, 0), (3, 1), (0, 1)):
        rc = oracle.lin_witness(hist(rows), prefill=[1], drain=[1, 5, 6], capacity=cap)[0]
        assert rc == want, cap
        assert check_linearizable(with_drain(rows, [1, 5, 6]), capacity=cap or None,
                                  prefill=[1])[0] == bool(want)


def test_full_is_effect_free():
    rows = [(0, OP_ENQ, ST_FULL, 9, 0, 1), (1, OP_DEQ, ST_EMPTY, 0, 2, 3)]
    rc, order, _ = oracle.lin_witness(hist(rows), capacity=4)
    assert rc == 1
    assert oracle.check_witness(hist(rows), order, capacity=4) == ""


def test_unsupported_duplicate_enqueue():
    rows = [(0, OP_ENQ, ST_OK, 5, 0, 1), (1, OP_ENQ, ST_OK, 5, 2, 3)]
    assert oracle.lin_witness(hist(rows), drain=[5, 5])[0] == oracle.LIN_UNSUPPORTED


def test_check_witness_rejects_bad_orders():
    """The witness check is pinned on its own: it rejects an order that breaks
    real time, one whose replay gives another answer, and a non-permutation."""
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 2, 2, 3),
            (1, OP_DEQ, ST_OK, 1, 4, 5), (1, OP_DEQ, ST_OK, 2, 6, 7)]
    h = hist(rows)
    good = [0, 1, 2, 3, 4]
    assert oracle.check_witness(h, good) == ""
    assert "real-time" in oracle.check_witness(h, [1, 0, 2, 3, 4])
    rows2 = [(0, OP_ENQ, ST_OK, 1, 0, 10), (0, OP_ENQ, ST_OK, 2, 0, 10),
             (1, OP_DEQ, ST_OK, 1, 11, 12), (1, OP_DEQ, ST_OK, 2, 13, 14)]
    h2 = hist(rows2)
    assert oracle.check_witness(h2, [0, 1, 2, 3, 4]) == ""
    assert "replay" in oracle.check_witness(h2, [1, 0, 2, 3, 4])
    assert "permutation" in oracle.check_witness(h, [0, 1, 2, 3])
    assert "permutation" in oracle.check_witness(h, [0, 1, 2, 2, 4])


def big_legal(seed, n, spread, p_enq=0.5, capacity=None, nprocs=None, prefill=0):
    """A legal sequential run of n operations whose linearization instants are
    10 apart, each interval stretched by up to `spread` on both sides (each
    lane's operations kept in program order by giving every operation its own
    lane unless nprocs is set, in which case lanes are disjoint in time)."""
    rng = np.random.default_rng(seed)
    q = collections.deque(range(1, prefill + 1))
    isenq = rng.random(n) < p_enq
    op = np.where(isenq, OP_ENQ, OP_DEQ).astype(np.uint8)
    st = np.zeros(n, np.uint8)
    val = np.zeros(n, np.uint64)
    nv = 1 << 20
    for i in range(n):
        if isenq[i]:
            val[i] = nv
            if capacity and len(q) >= capacity:
                st[i] = ST_FULL
            else:
                q.append(nv)
            nv += 1
        elif q:
            val[i] = q.popleft()
        else:
            st[i] = ST_EMPTY
    t = 10 * np.arange(1, n + 1, dtype=np.int64) + 10 ** 6
    call = t - rng.integers(0, spread, n)
    ret = t + rng.integers(0, spread, n)
    proc = np.arange(n) if nprocs is None else np.arange(n) % nprocs
    if nprocs is not None:
        # a lane's consecutive operations are nprocs instants apart: keep them disjoint
        half = 5 * nprocs
        call = np.maximum(call, t - half + 1)
        ret = np.minimum(ret, t + half - 1)
    h = oracle.History(proc, op, st, val, call.astype(np.uint64), ret.astype(np.uint64))
    return h, list(range(1, prefill + 1)), list(q)


@pytest.mark.parametrize("n,spread,cap,pre,p_enq", [
    (100000, 60, None, 0, 0.5),          # few overlaps
    (100000, 20000, None, 0, 0.5),       # each op overlaps ~4000 others
    (100000, 5000, 64, 32, 0.5),         # bounded, often FULL
    (100000, 5000, None, 0, 0.35),       # often EMPTY
])
def test_large_legal_history_found(n, spread, cap, pre, p_enq):
    h, prefill, drain = big_legal(7, n, spread, p_enq=p_enq, capacity=cap, prefill=pre)
    rc, order, info = oracle.lin_witness(h, prefill=prefill, drain=drain, capacity=cap or 0,
                                         width=2, budget=1000)
    assert rc == 1, info
    assert info["backtracks"] == 0
    assert oracle.check_witness(h, order, prefill=prefill, drain=drain, capacity=cap or 0) == ""


def test_large_history_with_lanes_found():
    h, prefill, drain = big_legal(8, 60000, 3000, nprocs=512, prefill=100)
    rc, order, _ = oracle.lin_witness(h, prefill=prefill, drain=drain, width=2, budget=1000)
    assert rc == 1
    assert oracle.check_witness(h, order, prefill=prefill, drain=drain) == ""


@pytest.mark.parametrize("mistake", ["swap", "empty", "drop"])
def test_large_history_planted_mistake_not_found(mistake):
    """A large history with one planted queue bug yields no witness."""
    h, prefill, drain = big_legal(9, 50000, 2000)
    d = np.where((h.op == OP_DEQ) & (h.st == ST_OK))[0]
    val, st = h.val.copy(), h.st.copy()
    a, b = d[len(d) // 3], d[2 * len(d) // 3]
    if mistake == "swap":                # two dequeues far apart return each other's item
        val[a], val[b] = val[b], val[a]
    elif mistake == "empty":             # an OK dequeue reports EMPTY; its item drained last
        drain = drain + [int(val[a])]
        st[a], val[a] = ST_EMPTY, 0
    else:                                # an item is lost: its dequeue reports EMPTY, no drain
        st[a], val[a] = ST_EMPTY, 0
    h2 = oracle.History(h.proc, h.op, st, val, h.call, h.ret)
    rc, _, _ = oracle.lin_witness(h2, prefill=prefill, drain=drain, width=2, budget=2000)
    assert rc != 1


def test_capacity_bounds_of_the_gpu_test_helper():
    """The necessary n-bounded conditions the GPU tests pair with a witness
    found at n + 1: three OK enqueues returned before any dequeue starts need
    3 slots; a dequeue of the first item starting before the third enqueue
    returns leaves 2; an item whose dequeue starts after two later enqueues
    returned needs itself plus those two."""
    import numpy as np

    import oracle
    from tests.gpu_util import capacity_bounds

    def hist(rows):
        p, o, s, v, c, r = (np.array(x) for x in zip(*rows))
        return oracle.History(p, o, s, v.astype(np.uint64), c, r)

    enq = [(0, 0, 0, 10, 0, 1), (1, 0, 0, 11, 2, 3), (2, 0, 0, 12, 4, 5)]
    assert capacity_bounds(hist(enq + [(3, 1, 0, 10, 6, 7)]), (), 2) == 3
    assert capacity_bounds(hist(enq + [(3, 1, 0, 10, 4.5, 7)]), (), 2) == 2
    # item 10 dequeued late, after 11 and 12 both started and returned behind it
    late = [(0, 0, 0, 10, 0, 1), (3, 1, 0, 11, 3.5, 3.8), (1, 0, 0, 11, 2, 3),
            (2, 0, 0, 12, 4, 5), (4, 1, 0, 10, 6, 7)]
    assert capacity_bounds(hist(late), (), 4) == 3
