"""Pins for the CPU oracle: every part is checked against something other than
itself -- hand-derived fixtures, closed forms, textbook/library routines, and
brute force on tiny inputs -- so that a dropped term, a wrong sign or index, or
a transposed operand in the oracle fails here.  CPU only."""
import collections
import itertools
import os
import random

import numpy as np
import pytest

import oracle
from oracle import History, OP_DEQ, OP_ENQ, ST_EMPTY, ST_FULL, ST_OK
from oracle.linearize import check_linearizable

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# O1/O2: sequential replay
# ---------------------------------------------------------------------------
def _load_fifo_fixture(name):
    ops, args, st, val = [], [], [], []
    capacity, prefill, residual = 0, [], []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "capacity":
            capacity = int(tok[1])
        elif tok[0] == "prefill":
            prefill = [int(x) for x in tok[1:]]
        elif tok[0] == "residual":
            residual = [int(x) for x in tok[1:]]
        else:
            ops.append(OP_ENQ if tok[0] == "E" else OP_DEQ)
            args.append(int(tok[1]))
            st.append({"OK": ST_OK, "EMPTY": ST_EMPTY, "FULL": ST_FULL}[tok[2]])
            val.append(int(tok[3]))
    return capacity, prefill, ops, args, st, val, residual


def test_replay_golden_fixture():
    cap, pre, ops, args, st_exp, val_exp, resid_exp = _load_fifo_fixture("fifo_small.txt")
    st, val, resid = oracle.fifo_replay(ops, args, capacity=cap, prefill=pre)
    assert st.tolist() == st_exp
    assert val.tolist() == val_exp
    assert resid.tolist() == resid_exp


def test_replay_closed_form_fill_then_drain():
    m = 1000
    ops = [OP_ENQ] * m + [OP_DEQ] * (m + 5)
    args = list(range(1, m + 1)) + [0] * (m + 5)
    st, val, resid = oracle.fifo_replay(ops, args)
    assert (st[:m] == ST_OK).all()
    assert val[m:2 * m].tolist() == list(range(1, m + 1))
    assert (st[2 * m:] == ST_EMPTY).all()
    assert len(resid) == 0


def test_replay_capacity_closed_form():
    n, extra = 64, 9
    ops = [OP_ENQ] * (n + extra) + [OP_DEQ] * n
    args = list(range(1, n + extra + 1)) + [0] * n
    st, val, resid = oracle.fifo_replay(ops, args, capacity=n)
    assert (st[:n] == ST_OK).all() and (st[n:n + extra] == ST_FULL).all()
    # FULL left no trace: the dequeues return exactly 1..n
    assert val[n + extra:].tolist() == list(range(1, n + 1))


@pytest.mark.parametrize("seed", range(20))
def test_replay_matches_library_deque(seed):
    """Against collections.deque (a textbook FIFO from the standard library)."""
    rng = random.Random(seed)
    cap = rng.choice([0, 1, 2, 5, 17])
    pre = [rng.randrange(1 << 40) for _ in range(rng.randrange(0, cap or 4))]
    m = 500
    ops = [rng.choice([OP_ENQ, OP_DEQ]) for _ in range(m)]
    args = [rng.randrange(1, 1 << 62) for _ in range(m)]
    q = collections.deque(pre)
    exp_st, exp_val = [], []
    for o, a in zip(ops, args):
        if o == OP_ENQ:
            if cap and len(q) >= cap:
                exp_st.append(ST_FULL); exp_val.append(a)
            else:
                q.append(a); exp_st.append(ST_OK); exp_val.append(a)
        else:
            if q:
                exp_st.append(ST_OK); exp_val.append(q.popleft())
            else:
                exp_st.append(ST_EMPTY); exp_val.append(0)
    st, val, resid = oracle.fifo_replay(ops, args, capacity=cap, prefill=pre)
    assert st.tolist() == exp_st
    assert val.tolist() == exp_val
    assert resid.tolist() == list(q)


def test_replay_conservation_invariant():
    rng = np.random.default_rng(3)
    m = 20000
    ops = rng.integers(0, 2, m).astype(np.uint8)
    args = np.arange(1, m + 1, dtype=np.uint64)
    st, val, resid = oracle.fifo_replay(ops, args, capacity=300, prefill=[7, 8])
    put = np.concatenate([[7, 8], args[(ops == OP_ENQ) & (st == ST_OK)]])
    out = np.concatenate([val[(ops == OP_DEQ) & (st == ST_OK)], resid])
    # FIFO: values leave in exactly the order they entered
    assert np.array_equal(put, out)


# ---------------------------------------------------------------------------
# O3: conservation
# ---------------------------------------------------------------------------
def test_conservation_catalogue():
    assert oracle.conservation([1, 2, 3], [3, 1, 2]) == {"lost": 0, "extra": 0, "dup_in": 0}
    assert oracle.conservation([1, 2, 3], [3, 1]) == {"lost": 1, "extra": 0, "dup_in": 0}
    assert oracle.conservation([1, 2, 3], [3, 1, 2, 2]) == {"lost": 0, "extra": 1, "dup_in": 0}
    assert oracle.conservation([1, 2, 3], [3, 1, 9]) == {"lost": 1, "extra": 1, "dup_in": 0}
    assert oracle.conservation([1, 1, 3], [1, 1, 3]) == {"lost": 0, "extra": 0, "dup_in": 1}
    assert oracle.conservation([], []) == {"lost": 0, "extra": 0, "dup_in": 0}


def test_conservation_against_counter():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 50, 2000).astype(np.uint64)
    b = rng.integers(0, 50, 2100).astype(np.uint64)
    ca, cb = collections.Counter(a.tolist()), collections.Counter(b.tolist())
    exp_lost = sum((ca - cb).values())
    exp_extra = sum((cb - ca).values())
    exp_dup = sum(v - 1 for v in ca.values())
    assert oracle.conservation(a, b) == {"lost": exp_lost, "extra": exp_extra, "dup_in": exp_dup}


# ---------------------------------------------------------------------------
# Helpers: legal-by-construction concurrent histories
# ---------------------------------------------------------------------------
def legal_history(rng, n_ops, n_procs, capacity=None, prefill=(), p_enq=0.5, spread=25):
    """Pick a legal sequential run, give each op a linearization instant 10*i,
    then stretch intervals around the instants (keeping each process's ops
    disjoint and in program order).  The result is linearizable by construction."""
    q = collections.deque(prefill)
    seq = []
    next_val = 1000
    for i in range(n_ops):
        if rng.random() < p_enq:
            if capacity is not None and len(q) >= capacity:
                seq.append((OP_ENQ, ST_FULL, next_val))
            else:
                q.append(next_val); seq.append((OP_ENQ, ST_OK, next_val))
            next_val += 1
        else:
            if q:
                seq.append((OP_DEQ, ST_OK, q.popleft()))
            else:
                seq.append((OP_DEQ, ST_EMPTY, 0))
    procs = [rng.randrange(n_procs) for _ in range(n_ops)]
    t = [10 * (i + 1) + 100 for i in range(n_ops)]
    call = [ti - rng.randint(0, spread) for ti in t]
    ret = [ti + rng.randint(0, spread) for ti in t]
    last = {}
    for i in range(n_ops):
        p = procs[i]
        if p in last:
            j = last[p]
            mid = (t[j] + t[i]) // 2
            ret[j] = min(ret[j], mid)
            call[i] = max(call[i], mid + 1)
        last[p] = i
    rows = [(procs[i], seq[i][0], seq[i][1], seq[i][2], call[i], ret[i]) for i in range(n_ops)]
    return rows, list(q)


def rows_to_history(rows):
    return History.from_rows(rows).sorted_by_proc()


# ---------------------------------------------------------------------------
# O5: exhaustive search, pinned by a plain permutation enumeration
# ---------------------------------------------------------------------------
def permutation_linearizable(rows, capacity=None, prefill=(), full="free"):
    """The definition spelled out: try every total order."""
    n = len(rows)
    for perm in itertools.permutations(range(n)):
        pos = {p: k for k, p in enumerate(perm)}
        if any(rows[a][5] < rows[b][4] and pos[a] > pos[b]
               for a in range(n) for b in range(n) if a != b):
            continue
        q = collections.deque(prefill)
        ok = True
        for i in perm:
            _, kind, st, val, _, _ = rows[i]
            if kind == OP_ENQ and st == ST_OK:
                if capacity is not None and len(q) >= capacity:
                    ok = False; break
                q.append(val)
            elif kind == OP_ENQ and st == ST_FULL:
                if full == "strict" and not (capacity is not None and len(q) == capacity):
                    ok = False; break
            elif st == ST_OK:
                if not q or q[0] != val:
                    ok = False; break
                q.popleft()
            else:
                if q:
                    ok = False; break
        if ok:
            return True
    return False


# Hand-built catalogue: (rows, linearizable?)  rows = (proc, op, st, val, call, ret)
CATALOGUE = [
    # sequential legal
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 2, 2, 3),
      (0, OP_DEQ, ST_OK, 1, 4, 5), (0, OP_DEQ, ST_OK, 2, 6, 7),
      (0, OP_DEQ, ST_EMPTY, 0, 8, 9)], True),
    # overlapping enqueues, dequeued in either order: both legal
    ([(0, OP_ENQ, ST_OK, 1, 0, 10), (1, OP_ENQ, ST_OK, 2, 0, 10),
      (2, OP_DEQ, ST_OK, 1, 11, 12), (2, OP_DEQ, ST_OK, 2, 13, 14)], True),
    ([(0, OP_ENQ, ST_OK, 1, 0, 10), (1, OP_ENQ, ST_OK, 2, 0, 10),
      (2, OP_DEQ, ST_OK, 2, 11, 12), (2, OP_DEQ, ST_OK, 1, 13, 14)], True),
    # dequeue returns an item whose enqueue is still in flight: legal
    ([(0, OP_ENQ, ST_OK, 1, 0, 20), (1, OP_DEQ, ST_OK, 1, 5, 10)], True),
    # non-overlapping enq 1 then enq 2, but deq 2 strictly before deq 1: VOrd
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 2, 2, 3),
      (1, OP_DEQ, ST_OK, 2, 4, 5), (1, OP_DEQ, ST_OK, 1, 6, 7)], False),
    # EMPTY while an item is definitely present: VWit
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_DEQ, ST_EMPTY, 0, 2, 3),
      (1, OP_DEQ, ST_OK, 1, 4, 5)], False),
    # EMPTY overlapping the enqueue: legal
    ([(0, OP_ENQ, ST_OK, 1, 0, 5), (1, OP_DEQ, ST_EMPTY, 0, 2, 3),
      (1, OP_DEQ, ST_OK, 1, 6, 7)], True),
    # duplicate delivery
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_DEQ, ST_OK, 1, 2, 3),
      (2, OP_DEQ, ST_OK, 1, 2, 3)], False),
    # fresh value
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_DEQ, ST_OK, 7, 2, 3)], False),
    # dequeue returns a value before its enqueue was called
    ([(1, OP_DEQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 1, 2, 3)], False),
    # the classic overlapping case: x enq, y enq overlapping deq -> y while x present
    ([(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_ENQ, ST_OK, 2, 2, 10),
      (2, OP_DEQ, ST_OK, 2, 3, 9)], False),
]


@pytest.mark.parametrize("rows,expected", CATALOGUE)
def test_bruteforce_catalogue(rows, expected):
    assert check_linearizable(rows)[0] is expected
    assert permutation_linearizable(rows) is expected


def test_bruteforce_witness_is_legal():
    rows = CATALOGUE[2][0]
    ok, order = check_linearizable(rows)
    assert ok
    st, val, _ = oracle.fifo_replay([rows[i][1] for i in order], [rows[i][3] for i in order])
    assert [int(v) for v in val] == [rows[i][3] if rows[i][1] == OP_ENQ or rows[i][2] == ST_OK
                                     else 0 for i in order]


@pytest.mark.parametrize("seed", range(60))
def test_bruteforce_matches_permutations(seed):
    """Random tiny arbitrary histories: the DFS equals the plain definition."""
    rng = random.Random(1000 + seed)
    n = rng.randint(1, 6)
    cap = rng.choice([None, 1, 2])
    rows = []
    for i in range(n):
        kind = rng.choice([OP_ENQ, OP_DEQ])
        st = rng.choice([ST_OK, ST_OK, ST_EMPTY if kind == OP_DEQ else ST_FULL])
        val = rng.randint(1, 3) if (kind == OP_ENQ or st == ST_OK) else 0
        c = rng.randint(0, 12)
        rows.append((i, kind, st, val, c, c + rng.randint(0, 8)))
    pre = [rng.randint(1, 3) for _ in range(rng.randint(0, 1))]
    for full in ("free", "strict"):
        assert check_linearizable(rows, capacity=cap, prefill=pre, full=full)[0] == \
            permutation_linearizable(rows, capacity=cap, prefill=pre, full=full)


def test_bruteforce_sequential_equals_replay():
    """A history with no overlap reduces to a replay of its real-time order."""
    rng = random.Random(7)
    for trial in range(200):
        n = rng.randint(1, 12)
        ops = [rng.choice([OP_ENQ, OP_DEQ]) for _ in range(n)]
        args = [rng.randint(1, 4) for _ in range(n)]
        st, val, _ = oracle.fifo_replay(ops, args, capacity=3)
        rows = [(0, ops[i], int(st[i]), int(val[i]), 2 * i, 2 * i + 1) for i in range(n)]
        assert check_linearizable(rows, capacity=3, full="strict")[0]
        # perturb one dequeue result: must become illegal (values are in 1..4)
        deqs = [i for i in range(n) if ops[i] == OP_DEQ and st[i] == ST_OK]
        if deqs:
            i = rng.choice(deqs)
            bad = list(rows[i]); bad[3] = int(val[i]) + 10
            rows2 = rows[:i] + [tuple(bad)] + rows[i + 1:]
            assert not check_linearizable(rows2, capacity=3, full="strict")[0]


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_accepts_legal_by_construction(seed):
    rng = random.Random(seed)
    cap = rng.choice([None, 2, 4])
    rows, _ = legal_history(rng, rng.randint(2, 14), rng.randint(1, 5), capacity=cap)
    assert check_linearizable(rows, capacity=cap, full="strict")[0]


# ---------------------------------------------------------------------------
# O6: violation scan
# ---------------------------------------------------------------------------
def scan(rows, prefill=(), drain=(), capacity=0):
    return oracle.violation_scan(rows_to_history(rows), prefill=prefill, drain=drain,
                                 capacity=capacity)


def test_scan_catalogue_patterns():
    # VOrd
    r = scan(CATALOGUE[4][0])
    assert r["order"] >= 1 and r["fresh"] == 0 and r["repeat"] == 0
    # VWit (item witness and count witness)
    r = scan(CATALOGUE[5][0])
    assert r["witness"] == 1 and r["witness_count"] == 1
    # duplicate
    assert scan(CATALOGUE[7][0])["repeat"] == 1
    # fresh value (never enqueued) and the enqueued 1 is lost
    r = scan(CATALOGUE[8][0])
    assert r["fresh"] == 1 and r["loss"] == 1
    # returned before the enqueue began
    assert scan(CATALOGUE[9][0])["fresh"] == 1
    # classic: y dequeued while x definitely present ahead of it -> VOrd with x
    # never dequeued (x counts as dequeued at +infinity) and x lost
    r = scan(CATALOGUE[10][0])
    assert r["order"] == 1 and r["loss"] == 1
    # the same history with x drained afterwards: still VOrd, no loss
    r = scan(CATALOGUE[10][0], drain=[1])
    assert r["order"] == 1 and r["loss"] == 0
    # legal ones are clean
    for rows, ok in CATALOGUE:
        if ok:
            assert oracle.all_zero(scan(rows)), rows


def test_scan_union_witness():
    """EMPTY over [4, 10]: value 1 is certainly present on (1, 7), value 2 on
    (5, 12).  Neither covers the EMPTY alone and the count bound is 0, but
    together they cover it: not linearizable (the exhaustive search agrees),
    and only the union witness finds it.  With value 2's enqueue ending at 8
    the instant 7.5 is uncovered and the history is legal."""
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_ENQ, ST_OK, 2, 2, 5),
            (2, OP_DEQ, ST_EMPTY, 0, 4, 10), (3, OP_DEQ, ST_OK, 1, 7, 8),
            (4, OP_DEQ, ST_OK, 2, 12, 13)]
    r = scan(rows)
    assert r["witness_union"] == 1 and r["witness"] == 0 and r["witness_count"] == 0
    assert sum(r.values()) == 1
    assert not check_linearizable(rows)[0]
    legal = [(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_ENQ, ST_OK, 2, 2, 8),
             (2, OP_DEQ, ST_EMPTY, 0, 4, 10), (3, OP_DEQ, ST_OK, 1, 7, 8),
             (4, OP_DEQ, ST_OK, 2, 12, 13)]
    assert oracle.all_zero(scan(legal))
    assert check_linearizable(legal)[0]
    # a value never dequeued covers to +infinity; a drained one up to its drain
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (2, OP_DEQ, ST_EMPTY, 0, 4, 10)]
    assert scan(rows, drain=[1])["witness_union"] == 1


def test_scan_return_code_covers_every_pattern():
    """The C entry point returns 1 exactly when some count is nonzero, the
    union witness (the last count) included: the history above that only the
    union witness flags must make it return 1."""
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_ENQ, ST_OK, 2, 2, 5),
            (2, OP_DEQ, ST_EMPTY, 0, 4, 10), (3, OP_DEQ, ST_OK, 1, 7, 8),
            (4, OP_DEQ, ST_OK, 2, 12, 13)]
    h = oracle.History.from_rows(rows)
    L = oracle.lib()
    out = np.zeros(len(oracle.VIOLATIONS), dtype=np.uint64)
    z = np.zeros(0, dtype=np.uint64)
    rc = L.orc_violation_scan(len(h), oracle._p(h.op), oracle._p(h.st), oracle._p(h.val),
                              oracle._p(h.call), oracle._p(h.ret), 0, oracle._p(z), 0,
                              oracle._p(z), 0, oracle._p(out))
    assert rc == 1 and int(out[-1]) == 1 and int(out[:-1].sum()) == 0
    legal = [(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_DEQ, ST_OK, 1, 2, 3)]
    h = oracle.History.from_rows(legal)
    rc = L.orc_violation_scan(len(h), oracle._p(h.op), oracle._p(h.st), oracle._p(h.val),
                              oracle._p(h.call), oracle._p(h.ret), 0, oracle._p(z), 0,
                              oracle._p(z), 0, oracle._p(out))
    assert rc == 0 and int(out.sum()) == 0


def test_scan_spurious_full():
    # capacity 2: one item in the queue, FULL answered: impossible
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (1, OP_ENQ, ST_FULL, 2, 2, 3)]
    assert scan(rows, capacity=2)["full"] == 1
    # two items present: FULL is fine
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 3, 2, 3),
            (1, OP_ENQ, ST_FULL, 2, 4, 5)]
    assert scan(rows, capacity=2, drain=[1, 3])["full"] == 0
    # one present plus one enqueue in flight: FULL may be legal (free index gone)
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (2, OP_ENQ, ST_OK, 3, 2, 9),
            (1, OP_ENQ, ST_FULL, 2, 4, 5)]
    assert scan(rows, capacity=2, drain=[1, 3])["full"] == 0
    # prefill counts as present
    rows = [(1, OP_ENQ, ST_FULL, 2, 4, 5)]
    assert scan(rows, capacity=2, prefill=[8, 9], drain=[8, 9])["full"] == 0
    assert scan(rows, capacity=3, prefill=[8, 9], drain=[8, 9])["full"] == 1


def test_scan_prefill_and_drain_order():
    # prefill [5, 6]; a dequeue returning 6 while 5 is never taken before it -> VOrd
    rows = [(0, OP_DEQ, ST_OK, 6, 0, 1)]
    assert scan(rows, prefill=[5, 6], drain=[5])["order"] == 1
    rows = [(0, OP_DEQ, ST_OK, 5, 0, 1)]
    assert oracle.all_zero(scan(rows, prefill=[5, 6], drain=[6]))
    # drain order matters: items must drain in enqueue order
    rows = [(0, OP_ENQ, ST_OK, 1, 0, 1), (0, OP_ENQ, ST_OK, 2, 2, 3)]
    assert oracle.all_zero(scan(rows, drain=[1, 2]))
    assert scan(rows, drain=[2, 1])["order"] == 1


@pytest.mark.parametrize("seed", range(40))
def test_scan_clean_on_legal_histories(seed):
    rng = random.Random(500 + seed)
    cap = rng.choice([None, 3, 8])
    pre = list(range(1, rng.randint(0, 3) + 1))
    rows, resid = legal_history(rng, rng.randint(1, 300), rng.randint(1, 12),
                                capacity=cap, prefill=pre)
    r = scan(rows, prefill=pre, drain=resid, capacity=cap or 0)
    assert oracle.all_zero(r), r


@pytest.mark.parametrize("seed", range(150))
def test_scan_is_sound_against_bruteforce(seed):
    """Whenever the scan flags a tiny history, the exhaustive search rejects it."""
    rng = random.Random(9000 + seed)
    cap = rng.choice([None, 2, 3])
    rows, resid = legal_history(rng, rng.randint(2, 9), rng.randint(1, 4), capacity=cap)
    # mutate: swap two dequeue results, turn an OK into EMPTY, drop/duplicate, shift time
    rows = [list(r) for r in rows]
    kind = rng.randrange(5)
    deqs = [i for i, r in enumerate(rows) if r[1] == OP_DEQ and r[2] == ST_OK]
    if kind == 0 and len(deqs) >= 2:
        a, b = rng.sample(deqs, 2)
        rows[a][3], rows[b][3] = rows[b][3], rows[a][3]
    elif kind == 1 and deqs:
        i = rng.choice(deqs); rows[i][2] = ST_EMPTY; resid = resid + [rows[i][3]]; rows[i][3] = 0
    elif kind == 2 and deqs:
        i = rng.choice(deqs); j = rng.choice(deqs); rows[j][3] = rows[i][3]
    elif kind == 3:
        i = rng.randrange(len(rows)); rows[i][4] = max(0, rows[i][4] + rng.randint(-30, 30))
        rows[i][5] = max(rows[i][4], rows[i][5] + rng.randint(-30, 30))
    else:
        e = [i for i, r in enumerate(rows) if r[1] == OP_DEQ and r[2] == ST_EMPTY]
        if e:
            i = rng.choice(e); rows[i][4] = max(0, rows[i][4] - 40)
    rows = [tuple(r) for r in rows]
    flags = scan(rows, drain=resid, capacity=cap or 0)
    lin = check_linearizable(rows + [(99, OP_DEQ, ST_OK, v, 10**6 + 2 * k, 10**6 + 2 * k + 1)
                                     for k, v in enumerate(resid)], capacity=cap)[0]
    flagged = any(v for k, v in flags.items() if k != "full")
    if flagged:
        assert not lin, (rows, flags)


# ---------------------------------------------------------------------------
# O4: per-producer order
# ---------------------------------------------------------------------------
def tok(p, s):
    return (p << 32) | (s + 1)


def test_producer_order_catalogue():
    ok_rows = [(0, OP_ENQ, ST_OK, tok(0, 0), 0, 1), (0, OP_ENQ, ST_OK, tok(0, 1), 2, 3),
               (1, OP_DEQ, ST_OK, tok(0, 0), 4, 5), (1, OP_DEQ, ST_OK, tok(0, 1), 6, 7)]
    assert oracle.all_zero(oracle.producer_order(rows_to_history(ok_rows)))
    # consumer sees seq 1 before seq 0
    bad = [(0, OP_ENQ, ST_OK, tok(0, 0), 0, 1), (0, OP_ENQ, ST_OK, tok(0, 1), 2, 3),
           (1, OP_DEQ, ST_OK, tok(0, 1), 4, 5), (1, OP_DEQ, ST_OK, tok(0, 0), 6, 7)]
    r = oracle.producer_order(rows_to_history(bad))
    assert r["consumer_order"] == 1 and r["realtime_order"] == 1
    # two consumers: deq(seq1) ends before deq(seq0) is called
    bad2 = [(0, OP_ENQ, ST_OK, tok(0, 0), 0, 1), (0, OP_ENQ, ST_OK, tok(0, 1), 2, 3),
            (1, OP_DEQ, ST_OK, tok(0, 1), 4, 5), (2, OP_DEQ, ST_OK, tok(0, 0), 6, 7)]
    r = oracle.producer_order(rows_to_history(bad2))
    assert r["consumer_order"] == 0 and r["realtime_order"] == 1
    # overlapping dequeues may finish in either order
    ok2 = [(0, OP_ENQ, ST_OK, tok(0, 0), 0, 1), (0, OP_ENQ, ST_OK, tok(0, 1), 2, 3),
           (1, OP_DEQ, ST_OK, tok(0, 1), 4, 8), (2, OP_DEQ, ST_OK, tok(0, 0), 5, 9)]
    assert oracle.all_zero(oracle.producer_order(rows_to_history(ok2)))
    # dequeued before it was enqueued
    bad3 = [(1, OP_DEQ, ST_OK, tok(3, 0), 0, 1), (0, OP_ENQ, ST_OK, tok(3, 0), 2, 3)]
    assert oracle.producer_order(rows_to_history(bad3))["deq_before_enq"] == 1
    # different producers never constrain each other
    ok3 = [(0, OP_ENQ, ST_OK, tok(0, 0), 0, 1), (2, OP_ENQ, ST_OK, tok(2, 0), 2, 3),
           (1, OP_DEQ, ST_OK, tok(2, 0), 4, 5), (1, OP_DEQ, ST_OK, tok(0, 0), 6, 7)]
    assert oracle.all_zero(oracle.producer_order(rows_to_history(ok3)))


@pytest.mark.parametrize("seed", range(20))
def test_producer_order_clean_on_legal(seed):
    rng = random.Random(77 + seed)
    rows, _ = legal_history(rng, 400, 8)
    # re-label values as producer tokens, in each producer's enqueue order
    cnt = collections.Counter()
    relabel = {}
    rows2 = []
    # enqueue program order per proc == order of linearization instants
    for r in sorted(rows, key=lambda r: (r[4] + r[5])):
        if r[1] == OP_ENQ and r[2] == ST_OK:
            relabel[r[3]] = tok(r[0], cnt[r[0]])
            cnt[r[0]] += 1
    for r in rows:
        v = relabel.get(r[3], 0) if (r[1] == OP_ENQ and r[2] == ST_OK) or \
            (r[1] == OP_DEQ and r[2] == ST_OK) else 0
        rows2.append((r[0], r[1], r[2], v, r[4], r[5]))
    assert oracle.all_zero(oracle.producer_order(rows_to_history(rows2)))


# ---------------------------------------------------------------------------
# O7: BFS
# ---------------------------------------------------------------------------
import workloads  # noqa: E402


def test_bfs_grid_is_manhattan_distance():
    R, C = 37, 53
    off, cols = workloads.grid_graph(R, C)
    root = 11 * C + 40
    lvl, nl, scanned = oracle.bfs(off, cols, root)
    r, c = np.divmod(np.arange(R * C), C)
    exp = np.abs(r - 11) + np.abs(c - 40)
    assert np.array_equal(lvl, exp.astype(np.uint32))
    assert nl == exp.max() + 1
    assert scanned == len(cols)


def test_bfs_corner_grid_levels():
    off, cols = workloads.grid_graph(64, 64)
    lvl, nl, _ = oracle.bfs(off, cols, 0)
    assert nl == 64 + 64 - 1


def test_bfs_path_star_and_unreachable():
    # path 0-1-2-...-9 plus isolated 10, 11
    src = np.arange(9); dst = np.arange(1, 10)
    off, cols = workloads._csr_from_pairs(12, src, dst)
    lvl, nl, _ = oracle.bfs(off, cols, 4)
    assert lvl[:10].tolist() == [4, 3, 2, 1, 0, 1, 2, 3, 4, 5]
    assert lvl[10] == 0xFFFFFFFF and lvl[11] == 0xFFFFFFFF
    assert nl == 6
    # star
    off, cols = workloads._csr_from_pairs(50, np.zeros(49, dtype=np.int64), np.arange(1, 50))
    lvl, nl, _ = oracle.bfs(off, cols, 7)
    assert lvl[7] == 0 and lvl[0] == 1 and (np.delete(lvl, [0, 7]) == 2).all() and nl == 3


@pytest.mark.parametrize("seed", range(8))
def test_bfs_matches_scipy_shortest_path(seed):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(seed)
    nv = 300
    ne = rng.integers(100, 900)
    off, cols = workloads._csr_from_pairs(nv, rng.integers(0, nv, ne), rng.integers(0, nv, ne))
    root = int(rng.integers(0, nv))
    lvl, _, _ = oracle.bfs(off, cols, root)
    A = csr_matrix((np.ones(len(cols)), cols.astype(np.int64), off.astype(np.int64)),
                   shape=(nv, nv))
    d = shortest_path(A, unweighted=True, indices=root)
    exp = np.where(np.isinf(d), 0xFFFFFFFF, d).astype(np.uint32)
    assert np.array_equal(lvl, exp)


def test_bfs_rmat_graph500_invariants():
    off, cols = workloads.rmat_graph(12, 16, seed=42)
    root = workloads.bfs_root(off, 42)
    lvl, nl, _ = oracle.bfs(off, cols, root)
    off64 = off.astype(np.int64)
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off64))
    lu, lv = lvl[rows].astype(np.int64), lvl[cols].astype(np.int64)
    reached_u = lu != 0xFFFFFFFF
    # every edge with a reached end has both ends reached, levels differ by <= 1
    assert np.array_equal(reached_u, lv != 0xFFFFFFFF)
    assert (np.abs(lu[reached_u] - lv[reached_u]) <= 1).all()
    # every reached non-root vertex has a neighbour one level closer
    parent_ok = np.zeros(len(lvl), dtype=bool)
    parent_ok[rows[(lv == lu - 1) & reached_u]] = True
    reached = lvl != 0xFFFFFFFF
    reached[root] = False
    assert parent_ok[reached].all()
    assert lvl[root] == 0


# ---------------------------------------------------------------------------
# Locked-queue baseline (measurement only): counts agree with the replay
# ---------------------------------------------------------------------------
def test_locked_queue_single_thread_matches_replay():
    roles = workloads.mix_roles(11, 1, 5000)
    oke, okd, sec = oracle.locked_queue_run(roles, 64, 32)
    tokens = workloads.mix_tokens(roles)
    st, val, _ = oracle.fifo_replay(roles[0], tokens[0], capacity=64,
                                    prefill=np.arange(1, 33))
    assert oke == int(((roles[0] == 0) & (st == ST_OK)).sum())
    assert okd == int(((roles[0] == 1) & (st == ST_OK)).sum())


def test_locked_queue_multithread_balance():
    roles = workloads.mix_roles(12, 4, 20000)
    oke, okd, sec = oracle.locked_queue_run(roles, 128, 64)
    assert 0 <= 64 + oke - okd <= 128
    assert sec > 0


# ---------------------------------------------------------------------------
# Multiset checksums (the conservation check of runs without a history)
# ---------------------------------------------------------------------------
def test_multiset_checksums_against_big_integers():
    rng = np.random.default_rng(17)
    v = rng.integers(0, 2**63, size=5000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    n, s1, s2 = oracle.multiset_checksums(v)
    ints = [int(x) for x in v]
    assert n == 5000
    assert s1 == sum(ints) % 2**64
    assert s2 == sum(x * x for x in ints) % 2**64


def test_multiset_checksums_closed_form_and_order_free():
    # 1..m: sum m(m+1)/2, sum of squares m(m+1)(2m+1)/6 (no wrap at this size)
    m = 100000
    v = np.arange(1, m + 1, dtype=np.uint64)
    assert oracle.multiset_checksums(v) == (m, m * (m + 1) // 2, m * (m + 1) * (2 * m + 1) // 6)
    rng = np.random.default_rng(3)
    assert oracle.multiset_checksums(rng.permutation(v)) == oracle.multiset_checksums(v)
    # a duplicate in place of another item changes S1 (here) or S2
    w = v.copy()
    w[10] = w[11]
    assert oracle.multiset_checksums(w) != oracle.multiset_checksums(v)
    assert oracle.multiset_checksums([]) == (0, 0, 0)


def test_mix_tokens_from_counts():
    toks = oracle.mix_tokens_from_counts([2, 0, 3], lane0=5)
    want = [(5 << 32) | 1, (5 << 32) | 2, (7 << 32) | 1, (7 << 32) | 2, (7 << 32) | 3]
    assert toks.tolist() == want
    assert oracle.mix_tokens_from_counts([]).size == 0
