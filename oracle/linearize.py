"""Exhaustive linearizability search for small queue histories (oracle part O5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition (Herlihy and Wing's linearizability, as the paper checks it in
Section IV): a history is linearizable iff its operations can be placed in one
total order that (a) keeps every real-time precedence -- if x returned before y
was called, x comes first -- and (b) is a legal run of the sequential FIFO
model: an enqueue appends its value; a dequeue returns the head, or EMPTY when
the state is empty.

The search is the Wing-Gong/Lowe depth-first search: repeatedly choose an
operation none of whose real-time predecessors is still pending, apply the
sequential model, and backtrack on an illegal step; visited (remaining set,
queue state) pairs are memoised.  Exponential, for histories of ~20 ops.

FULL answers: with ``full="free"`` a FULL enqueue is an effect-free step legal
in any state (the outer queue may run out of free indices while items are in
flight, so FULL is not tied to the linearized size); with ``full="strict"`` it
is legal only when the state holds ``capacity`` items.  An OK enqueue is always
illegal in a state holding ``capacity`` items (when a capacity is given).

Equal timestamps count as overlap: x precedes y only if x.ret < y.call.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

OP_ENQ, OP_DEQ = 0, 1
ST_OK, ST_EMPTY, ST_FULL = 0, 1, 2

Op = Tuple[int, int, int, int, int, int]  # (proc, op, st, val, call, ret)


def _step(state: Tuple[int, ...], o: Op, capacity: Optional[int], full: str):
    """Apply one operation to the sequential FIFO; None if illegal."""
    _, kind, st, val, _, _ = o
    if kind == OP_ENQ:
        if st == ST_OK:
            if capacity is not None and len(state) >= capacity:
                return None
            return state + (val,)
        if st == ST_FULL:
            if full == "free":
                return state
            if capacity is not None and len(state) == capacity:
                return state
            return None
        return None
    if st == ST_OK:
        if state and state[0] == val:
            return state[1:]
        return None
    if st == ST_EMPTY:
        return state if not state else None
    return None


def check_linearizable(ops: Sequence[Op], capacity: Optional[int] = None,
                       prefill: Iterable[int] = (), full: str = "free"
                       ) -> Tuple[bool, Optional[List[int]]]:
    """Returns (linearizable, witness order as indices into ops, or None)."""
    ops = list(ops)
    n = len(ops)
    if n > 40:
        raise ValueError("exhaustive search is meant for small histories")
    # pred[i]: bitmask of ops that really precede op i.
    pred = [0] * n
    for i in range(n):
        for j in range(n):
            if i != j and ops[j][5] < ops[i][4]:
                pred[i] |= 1 << j
    full_mask = (1 << n) - 1
    dead = set()
    order: List[int] = []

    def dfs(done: int, state: Tuple[int, ...]) -> bool:
        if done == full_mask:
            return True
        key = (done, state)
        if key in dead:
            return False
        for i in range(n):
            bit = 1 << i
            if done & bit or (pred[i] & ~done):
                continue
            nxt = _step(state, ops[i], capacity, full)
            if nxt is None:
                continue
            order.append(i)
            if dfs(done | bit, nxt):
                return True
            order.pop()
        dead.add(key)
        return False

    ok = dfs(0, tuple(prefill))
    return ok, (list(order) if ok else None)
