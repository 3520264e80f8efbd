"""Helpers for the GPU parity tests: run the HIP path through the C ABI, turn
recorded histories into oracle inputs, and apply the oracle's checks."""
from __future__ import annotations

import numpy as np

import oracle


def torch():
    import torch as t
    return t


def u64(t):
    """torch int64 CUDA/CPU tensor -> numpy uint64."""
    return t.cpu().numpy().view(np.uint64)


def drain_fifo(q, max_items: int):
    """Sequential drain by one lane (FIFO order), via the scripted driver."""
    import paper_2606_01693_amd as gq
    T = torch()
    k = max_items + 1
    ops = T.ones(k, dtype=T.uint8, device="cuda")
    args = T.zeros(k, dtype=T.int64, device="cuda")
    pauses = T.zeros(k, dtype=T.int16, device="cuda")
    n_ops = T.tensor([k], dtype=T.int32, device="cuda")
    h = gq.History(1, k)
    q.run_script(1, False, ops, args, pauses, n_ops, k, h)
    T.cuda.synchronize()
    proc, op, st, val, call, ret, _ = h.to_numpy()
    ok = st == gq.GQ_OK
    first_empty = int(np.argmin(ok)) if not ok.all() else len(ok)
    assert not ok[first_empty:].any(), "an OK dequeue after EMPTY in a sequential drain"
    assert first_empty < k, "drain did not reach EMPTY"
    return val[:first_empty].copy()


def prefill(q, items):
    """Enqueue `items` in list order (one lane, sequentially), so the oracle
    may take them as the queue's initial contents in that order; a batch
    enqueue leaves the order within the batch unspecified."""
    T = torch()
    if len(items) == 0:
        return
    t = T.tensor(np.asarray(items, dtype=np.uint64).view(np.int64), device="cuda")
    # one lane enqueues them in list order
    ops = T.zeros(len(items), dtype=T.uint8, device="cuda")
    pauses = T.zeros(len(items), dtype=T.int16, device="cuda")
    n_ops = T.tensor([len(items)], dtype=T.int32, device="cuda")
    import paper_2606_01693_amd as gq
    h = gq.History(1, len(items))
    q.run_script(1, False, ops, t, pauses, n_ops, len(items), h)
    T.cuda.synchronize()
    _, _, s, _, _, _, _ = h.to_numpy()
    assert (s == gq.GQ_OK).all()


def history(h) -> tuple:
    proc, op, st, val, call, ret, overflow = h.to_numpy()
    return oracle.History(proc, op, st, val, call, ret), overflow


def assert_clean(rep: dict, hist: oracle.History = None, drain=(), prefill=(), tag="case"):
    """Fail with the full report; keep the failing history for offline study
    (under gpurun_out/, which GPU runs bring back)."""
    if all(v == 0 for v in rep.values()):
        return
    if hist is not None:
        import os
        os.makedirs("gpurun_out", exist_ok=True)
        np.savez_compressed(os.path.join("gpurun_out", f"fail_{tag}.npz"), proc=hist.proc,
                            op=hist.op, st=hist.st, val=hist.val, call=hist.call,
                            ret=hist.ret, drain=np.asarray(drain, dtype=np.uint64),
                            prefill=np.asarray(prefill, dtype=np.uint64))
    import pytest
    pytest.fail("oracle report: " + ", ".join(f"{k}={v}" for k, v in rep.items()))


# Histories up to this many operations also get a linearization witness
# (O10) unless a test asks for it at any size.
WITNESS_MAX_OPS = 1 << 24


def capacity_bounds(hist: oracle.History, prefill=(), capacity=0) -> int:
    """Two necessary conditions of an n-bounded FIFO linearization, counted
    from the stamps alone: (a) at no enqueue's return do more than n items
    have to be present (prefill + OK enqueues returned by then - OK dequeues
    called by then); (b) for no item A do more than n items have to be
    present together at A's dequeue (A plus the OK enqueues that start after
    A's enqueue returns and return before A's dequeue is called: they follow
    A, so they leave after it).  Returns the larger of the two counts."""
    op, st = np.asarray(hist.op), np.asarray(hist.st)
    val = np.asarray(hist.val, dtype=np.uint64)
    call, ret = np.asarray(hist.call, dtype=np.int64), np.asarray(hist.ret, dtype=np.int64)
    eok = (op == 0) & (st == 0)
    dok = (op == 1) & (st == 0)
    e_ret = np.sort(ret[eok])
    d_call = np.sort(call[dok])
    a = len(prefill) + np.arange(1, len(e_ret) + 1) - np.searchsorted(d_call, e_ret, side="right")
    worst = int(a.max()) if len(a) else 0
    deq_call = dict(zip(val[dok].tolist(), call[dok].tolist()))
    ec, er = call[eok], ret[eok]
    by_call = np.argsort(ec)
    ec_s, er_s = ec[by_call], er[by_call]
    for v, ra in zip(val[eok].tolist(), er.tolist()):
        cd = deq_call.get(v)
        if cd is None:
            continue
        later = er_s[np.searchsorted(ec_s, ra, side="right"):]
        worst = max(worst, 1 + int((later < cd).sum()))
    return worst


def witness_report(hist: oracle.History, drain, prefill=(), capacity=0) -> dict:
    """O10: a linearization of the whole history (with the sequential drain
    and its final EMPTY appended), found by the witness search and confirmed
    by the independent replay check.  lin_no_witness = 1 when none was found
    within the search's budget (the search is complete for a found witness
    only; O6 says whether the history is provably wrong).
    A history that sits at its capacity for long stretches (a near-full
    producer/consumer run) can leave the search undecided at capacity n: its
    greedy choice of the next enqueue can fill the last slot with an item
    whose dequeue starts late.  Then a witness at capacity n + 1 is accepted
    together with the two necessary n-bounded conditions of capacity_bounds
    (the queue holds at most n indices by construction)."""
    rc, order, info = oracle.lin_witness(hist, prefill=prefill, drain=drain, capacity=capacity,
                                         width=2, budget=10000)
    bad = ""
    if rc == 1:
        bad = oracle.check_witness(hist, order, prefill=prefill, drain=drain, capacity=capacity)
    elif rc == -1 and capacity:
        rc1, order1, info1 = oracle.lin_witness(hist, prefill=prefill, drain=drain,
                                                capacity=capacity + 1, width=2, budget=10000)
        bound = capacity_bounds(hist, prefill, capacity)
        if rc1 == 1 and bound <= capacity:
            bad = oracle.check_witness(hist, order1, prefill=prefill, drain=drain,
                                       capacity=capacity + 1)
            print(f"[witness] undecided at capacity {capacity} ({info}); witness at "
                  f"{capacity + 1}, necessary bound {bound}, check={bad!r}", flush=True)
            return {"lin_no_witness": 0, "lin_witness_check": int(bool(bad))}
    if rc != 1 or bad:
        print(f"[witness] rc={rc} info={info} check={bad!r}", flush=True)
    return {"lin_no_witness": int(rc != 1), "lin_witness_check": int(bool(bad))}


def check_history(hist: oracle.History, drain, prefill=(), capacity=0, token_shift=32,
                  producer_order=True, witness=None):
    """Conservation + per-producer order + violation scan, and a linearization
    witness (O10) for histories of at most WITNESS_MAX_OPS operations (witness
    True/False forces it on/off).  Returns a report dict; every entry must be
    zero."""
    put = np.concatenate([np.asarray(prefill, dtype=np.uint64), hist.enq_ok()])
    out = np.concatenate([hist.deq_ok(), np.asarray(drain, dtype=np.uint64)])
    rep = {}
    rep.update({"cons_" + k: v for k, v in oracle.conservation(put, out).items()})
    if producer_order:
        rep.update({"po_" + k: v for k, v in oracle.producer_order(hist, token_shift).items()})
    rep.update({"v_" + k: v for k, v in
                oracle.violation_scan(hist, prefill=prefill, drain=drain,
                                      capacity=capacity).items()})
    if witness is None:
        witness = len(hist) <= WITNESS_MAX_OPS
    if witness:
        rep.update(witness_report(hist, drain, prefill=prefill, capacity=capacity))
    return rep
