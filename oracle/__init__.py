"""CPU oracle for the concurrent-queue hot path.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the HIP queues: it loads its
own C library (gq_oracle.c, built with gcc by ``build()``) and a pure-Python
exhaustive linearizability search (linearize.py) and a linearization witness
search for large histories (gq_linsearch.c, in the same library).

What it checks is the paper's correctness statement: histories are
linearizable with respect to the sequential FIFO model (Section IV), and every
token is delivered exactly once and in per-producer order (Section IV, device
FIFO conformance).  BFS levels are checked against a sequential queue BFS
(Section V-B).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from .linearize import check_linearizable  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gq_oracle.c")
_SRC_LIN = os.path.join(_HERE, "gq_linsearch.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OP_ENQ, OP_DEQ = 0, 1
ST_OK, ST_EMPTY, ST_FULL = 0, 1, 2


def build() -> str:
    """Compile the oracle's C part with gcc (always rebuilds)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
           _SRC, _SRC_LIN, "-o", _LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        U64 = ctypes.c_uint64
        L.orc_fifo_replay.restype = ctypes.c_int64
        L.orc_fifo_replay.argtypes = [U64, P, P, U64, U64, P, P, P, P]
        L.orc_conservation.restype = ctypes.c_int
        L.orc_conservation.argtypes = [U64, P, U64, P, P]
        L.orc_producer_order.restype = ctypes.c_int
        L.orc_producer_order.argtypes = [U64, P, P, P, P, P, P, ctypes.c_uint32, P]
        L.orc_violation_scan.restype = ctypes.c_int
        L.orc_violation_scan.argtypes = [U64, P, P, P, P, P, U64, P, U64, P, U64, P]
        L.orc_bfs.restype = ctypes.c_int64
        L.orc_bfs.argtypes = [U64, P, P, ctypes.c_uint32, P, P]
        L.orc_lin_witness.restype = ctypes.c_int
        L.orc_lin_witness.argtypes = [U64, P, P, P, P, P, U64, P, U64, P, ctypes.c_int, U64, U64,
                                      ctypes.c_uint32, P, P]
        L.orc_locked_queue_run.restype = ctypes.c_int
        L.orc_locked_queue_run.argtypes = [ctypes.c_uint32, U64, P, U64, U64, P,
                                           ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _u64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def _u8(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


# ----------------------------------------------------------------------------
# History container
# ----------------------------------------------------------------------------
@dataclass
class History:
    """Struct-of-arrays history, grouped by proc, program order inside a proc."""
    proc: np.ndarray   # uint32
    op: np.ndarray     # uint8  (0 enq, 1 deq)
    st: np.ndarray     # uint8  (0 OK, 1 EMPTY, 2 FULL)
    val: np.ndarray    # uint64
    call: np.ndarray   # uint64
    ret: np.ndarray    # uint64

    def __post_init__(self):
        self.proc = np.ascontiguousarray(self.proc, dtype=np.uint32)
        self.op = _u8(self.op)
        self.st = _u8(self.st)
        self.val = _u64(self.val)
        self.call = _u64(self.call)
        self.ret = _u64(self.ret)

    def __len__(self):
        return int(self.op.shape[0])

    @staticmethod
    def from_rows(rows):
        """rows: iterable of (proc, op, st, val, call, ret)."""
        rows = list(rows)
        if not rows:
            z = np.zeros(0)
            return History(z, z, z, z, z, z)
        cols = list(zip(*rows))
        return History(*[np.array(c) for c in cols])

    def sorted_by_proc(self) -> "History":
        """Stable reorder so each proc's ops are contiguous (keeps order)."""
        o = np.argsort(self.proc, kind="stable")
        return History(self.proc[o], self.op[o], self.st[o], self.val[o],
                       self.call[o], self.ret[o])

    def enq_ok(self):
        return self.val[(self.op == OP_ENQ) & (self.st == ST_OK)]

    def deq_ok(self):
        return self.val[(self.op == OP_DEQ) & (self.st == ST_OK)]


# ----------------------------------------------------------------------------
# O1/O2 sequential replay
# ----------------------------------------------------------------------------
def fifo_replay(ops, args, capacity: int = 0, prefill=()):
    """Replay a total order through the bounded sequential FIFO.

    Returns (status uint8[m], values uint64[m], residual uint64[]).
    """
    op = _u8(ops)
    arg = _u64(args)
    pre = _u64(prefill)
    m = op.shape[0]
    st = np.zeros(m, dtype=np.uint8)
    val = np.zeros(m, dtype=np.uint64)
    resid = np.zeros(m + pre.shape[0] + 1, dtype=np.uint64)
    n = lib().orc_fifo_replay(m, _p(op), _p(arg), capacity, pre.shape[0], _p(pre),
                              _p(st), _p(val), _p(resid))
    if n < 0:
        raise MemoryError("orc_fifo_replay")
    return st, val, resid[:n].copy()


# ----------------------------------------------------------------------------
# O3 conservation
# ----------------------------------------------------------------------------
def conservation(put_in, taken_out):
    """Returns dict(lost, extra, dup_in); all zero iff the multisets match."""
    a = _u64(put_in)
    b = _u64(taken_out)
    out = np.zeros(3, dtype=np.uint64)
    rc = lib().orc_conservation(a.shape[0], _p(a), b.shape[0], _p(b), _p(out))
    if rc < 0:
        raise MemoryError("orc_conservation")
    return {"lost": int(out[0]), "extra": int(out[1]), "dup_in": int(out[2])}


def multiset_checksums(values):
    """(count, S1, S2) of a multiset of 64-bit items: S1 and S2 are the sums of
    v and of v * v taken modulo 2^64 (wrapping arithmetic).  Equal multisets
    have equal checksums; the device drivers report the same three numbers
    for the items they moved, so conservation (Section IV, each token exactly
    once) can be checked where no per-operation history is recorded."""
    v = _u64(values)
    with np.errstate(over="ignore"):
        return int(v.shape[0]), int(v.sum(dtype=np.uint64)), int((v * v).sum(dtype=np.uint64))


def mix_tokens_from_counts(lane_enq, lane0: int = 0):
    """The tokens a run's lanes enqueued successfully, given each lane's count
    of successful enqueues: lane g's j-th one carries (g << 32) | (j + 1)
    (the Section IV token format)."""
    cnt = np.asarray(lane_enq, dtype=np.int64)
    lanes = np.repeat(np.arange(lane0, lane0 + cnt.shape[0], dtype=np.uint64), cnt)
    within = np.arange(int(cnt.sum()), dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    return (lanes << np.uint64(32)) | (within + 1).astype(np.uint64)


# ----------------------------------------------------------------------------
# O4 per-producer order
# ----------------------------------------------------------------------------
def producer_order(h: History, shift: int = 32):
    out = np.zeros(3, dtype=np.uint64)
    rc = lib().orc_producer_order(len(h), _p(h.proc), _p(h.op), _p(h.st), _p(h.val),
                                  _p(h.call), _p(h.ret), shift, _p(out))
    if rc < 0:
        raise MemoryError("orc_producer_order")
    return {"consumer_order": int(out[0]), "realtime_order": int(out[1]),
            "deq_before_enq": int(out[2])}


# ----------------------------------------------------------------------------
# O6 violation scan
# ----------------------------------------------------------------------------
VIOLATIONS = ("fresh", "repeat", "order", "witness", "witness_count", "full", "loss",
              "witness_union")


def violation_scan(h: History, prefill=(), drain=(), capacity: int = 0):
    pre = _u64(prefill)
    dr = _u64(drain)
    out = np.zeros(len(VIOLATIONS), dtype=np.uint64)
    rc = lib().orc_violation_scan(len(h), _p(h.op), _p(h.st), _p(h.val), _p(h.call),
                                  _p(h.ret), pre.shape[0], _p(pre), dr.shape[0], _p(dr),
                                  capacity, _p(out))
    if rc < 0:
        raise MemoryError("orc_violation_scan")
    rep = {k: int(v) for k, v in zip(VIOLATIONS, out)}
    if rc != int(any(rep.values())):
        raise AssertionError(f"orc_violation_scan returned {rc} with counts {rep}")
    return rep


# ----------------------------------------------------------------------------
# O10 linearization witness search
# ----------------------------------------------------------------------------
LIN_FOUND, LIN_NONE, LIN_UNKNOWN, LIN_UNSUPPORTED = 1, 0, -1, -2


def lin_witness(h: History, prefill=(), drain=(), drain_ends_empty: bool = True,
                capacity: int = 0, budget: int = 1 << 62, width: int = 0):
    """Search for a linearization of the history (Section IV).

    Returns (code, order, info): code 1 = found (order: operation indices in
    linearization order; len(h) + j is the j-th drained item's dequeue and
    len(h) + len(drain) the drain's final EMPTY), 0 = none exists (complete
    search: width 0 or no branch cut short), -1 = undecided within the budget
    or width, -2 = unsupported history (an item enqueued twice, ...).
    width 0 is the exhaustive, memoised search; width w > 0 keeps the w best
    candidates per branch (for large histories); `budget` bounds the dead
    ends (backtracks) before the search gives up."""
    pre = _u64(prefill)
    dr = _u64(drain)
    m = len(h)
    M = m + dr.shape[0] + (1 if drain_ends_empty else 0)
    order = np.zeros(max(M, 1), dtype=np.uint64)
    info = np.zeros(4, dtype=np.uint64)
    rc = lib().orc_lin_witness(m, _p(h.op), _p(h.st), _p(h.val), _p(h.call), _p(h.ret),
                               pre.shape[0], _p(pre), dr.shape[0], _p(dr),
                               1 if drain_ends_empty else 0, capacity, budget, width,
                               _p(order), _p(info))
    if rc == -3:
        raise MemoryError("orc_lin_witness")
    return rc, (order[:M].astype(np.int64) if rc == 1 else None), {
        "branches": int(info[0]), "backtracks": int(info[1]), "longest_prefix": int(info[2]),
        "dead_end_op": int(info[3]) if int(info[3]) != (1 << 64) - 1 else -1}


def check_witness(h: History, order, prefill=(), drain=(), drain_ends_empty: bool = True,
                  capacity: int = 0) -> str:
    """Independent check of a claimed linearization: it must be a permutation
    of all operations (history, drained dequeues, final EMPTY), keep real-time
    precedence (no operation placed after one that was called after it
    returned), and replay through the sequential FIFO (O2) with every
    answer reproduced; FULL answers are effect-free and are left out of the
    replay.  Returns "" when it holds, else what failed."""
    dr = _u64(drain)
    m = len(h)
    M = m + dr.shape[0] + (1 if drain_ends_empty else 0)
    order = np.asarray(order, dtype=np.int64)
    if order.shape[0] != M or not np.array_equal(np.sort(order), np.arange(M)):
        return "not a permutation of the operations"
    tmax = int(max(h.call.max(initial=0), h.ret.max(initial=0)))
    extra = M - m
    call = np.concatenate([h.call, np.array([tmax + 1 + 2 * j for j in range(extra)],
                                            dtype=np.uint64)])
    ret = np.concatenate([h.ret, np.array([tmax + 2 + 2 * j for j in range(extra)],
                                          dtype=np.uint64)])
    op = np.concatenate([h.op, np.full(extra, OP_DEQ, dtype=np.uint8)])
    st = np.concatenate([h.st, np.array([ST_OK] * dr.shape[0] + [ST_EMPTY] * (extra - dr.shape[0]),
                                        dtype=np.uint8)])
    val = np.concatenate([h.val, dr, np.zeros(extra - dr.shape[0], dtype=np.uint64)])
    # real time: the largest call placed so far must not exceed any later return
    c = call[order]
    r = ret[order]
    before = np.maximum.accumulate(c)[:-1]  # largest call among the positions before k
    if np.any(before > r[1:]):
        k = int(np.argmax(before > r[1:])) + 1
        return f"real-time order broken at position {k}"
    keep = order[st[order] != ST_FULL]
    rs, rv, _ = fifo_replay(op[keep], val[keep], capacity=capacity, prefill=prefill)
    if not np.array_equal(rs, st[keep]):
        k = int(np.argmax(rs != st[keep]))
        return f"replay status differs at position {k}"
    okd = (op[keep] == OP_DEQ) & (st[keep] == ST_OK)
    if not np.array_equal(rv[okd], val[keep][okd]):
        return "replay dequeue values differ"
    return ""


def all_zero(d: dict) -> bool:
    return all(v == 0 for v in d.values())


# ----------------------------------------------------------------------------
# O7 BFS
# ----------------------------------------------------------------------------
def bfs(offsets, cols, root: int):
    """Returns (levels uint32[nv], n_levels, edges_scanned)."""
    off = _u64(offsets)
    c = np.ascontiguousarray(np.asarray(cols, dtype=np.uint32))
    nv = off.shape[0] - 1
    lvl = np.zeros(nv, dtype=np.uint32)
    scanned = np.zeros(1, dtype=np.uint64)
    nl = lib().orc_bfs(nv, _p(off), _p(c), root, _p(lvl), _p(scanned))
    if nl < 0:
        raise ValueError("orc_bfs failed")
    return lvl, int(nl), int(scanned[0])


# ----------------------------------------------------------------------------
# Host locked-queue baseline
# ----------------------------------------------------------------------------
def locked_queue_run(roles: np.ndarray, capacity: int, prefill: int):
    """roles: uint8 [threads, ops]. Returns (ok_enq, ok_deq, seconds)."""
    r = _u8(roles)
    threads, ops = r.shape
    out = np.zeros(2, dtype=np.uint64)
    sec = ctypes.c_double(0.0)
    rc = lib().orc_locked_queue_run(threads, ops, _p(r), capacity, prefill, _p(out),
                                    ctypes.byref(sec))
    if rc != 0:
        raise MemoryError("orc_locked_queue_run")
    return int(out[0]), int(out[1]), float(sec.value)
