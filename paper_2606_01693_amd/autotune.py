"""Autotuner for the queue drivers: grid search with a JSON cache.

Two searches, each timing real launches on the current device with HIP events
(median of `reps` after one warmup) and keeping the fastest configuration:

* ``tune_mix`` -- one queue under the mixed 50/50 workload at a fixed number of
  operation attempts: ticket group (64 = per-wavefront WaveFAA up to 1024 =
  one FAA per workgroup), lane count (the workgroup count), slot layout, ring
  capacity (the workload's capacity times a factor, the items in flight
  unchanged) and, for G-WFQ / G-WFQ-YMC, patience.  A configuration counts
  only if its runs conserve the items: the kernel's multiset checksums of
  what went in (prefill, enqueues) equal those of what came out (dequeues,
  the drained remainder).
* ``tune_multi`` -- the many-queue persistent launch: wavefronts given to each
  queue per 256 of its slots, with the work per queue fixed (4n operations in
  the 50/50 mix, the many-queue configuration), so more lanes means fewer
  operations per lane.

* ``tune_prodcons`` -- G-WFQ's slow-path knobs under an imbalanced
  producer/consumer run (the C3 shape): patience (enqueue, dequeue) and help
  delay D.  A run counts only when every item went through with the
  multiset checksums equal; the fastest such configuration wins.

Results are cached in a JSON file keyed by device architecture, queue kind
and sizes; a cached key is returned without measuring unless ``force``.  The
measuring function can be replaced (``measure=``), which is how the search
and cache logic are tested without a GPU.
"""
from __future__ import annotations

import itertools
import json
import os
from dataclasses import asdict, dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class TuneResult:
    key: str
    best: Dict
    best_ms: float
    best_mops: float
    table: List[Dict] = field(default_factory=list)


def _load(path: str) -> Dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path: str, key: str, res: TuneResult) -> None:
    if not path:
        return
    data = _load(path)
    data[key] = asdict(res)
    tmp = path + ".tmp"
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached(path: str, key: str) -> Optional[TuneResult]:
    d = _load(path).get(key)
    return TuneResult(**d) if d else None


def _search(key: str, candidates: List[Dict], measure: Callable[[Dict], tuple],
            cache_path: str, force: bool) -> TuneResult:
    if not force:
        hit = cached(cache_path, key)
        if hit is not None:
            return hit
    table = []
    for cand in candidates:
        try:
            ms, ok_ops = measure(cand)
        except Exception as e:  # a configuration the library refuses (cycle bound, residency)
            table.append(dict(cand, error=str(e)))
            continue
        table.append(dict(cand, ms=ms, mops=ok_ops / (ms * 1e-3) / 1e6))
    good = [t for t in table if "ms" in t]
    if not good:
        raise RuntimeError(f"autotune {key}: every configuration failed: {table}")
    best = max(good, key=lambda t: t["mops"])
    res = TuneResult(key=key, best={k: v for k, v in best.items() if k not in ("ms", "mops")},
                     best_ms=best["ms"], best_mops=best["mops"], table=table)
    _store(cache_path, key, res)
    return res


def _device_arch() -> str:
    from . import device_info
    return device_info()["arch"].split(":")[0]


def _time_ms(torch, fn, reps: int) -> float:
    fn()  # warmup
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    return float(np.median(ms))


def tune_mix(kind: str, capacity: int, total_ops: int = 1 << 24,
             ticket_groups=(64, 256, 512, 1024), lanes_options=(1 << 17, 1 << 18, 1 << 19),
             slot_modes=("linear", "remap"), capacity_factors=(1, 2, 4),
             patience_options=(None,), reps: int = 3,
             cache_path: str = "", force: bool = False,
             measure: Callable[[Dict], tuple] = None) -> TuneResult:
    """Fastest configuration for `total_ops` mixed 50/50 attempts on one queue
    holding capacity/2 items (uint64), its ring `capacity` times a factor."""
    key = (f"mix/{_arch_or('any', measure)}/{kind}/cap{capacity}/ops{total_ops}"
           f"/f{'-'.join(str(f) for f in capacity_factors)}")
    cands = [dict(ticket_group=tg, lanes=l, slot_mode=sm, capacity_factor=f, patience=p)
             for tg, l, sm, f, p in itertools.product(ticket_groups, lanes_options, slot_modes,
                                                      capacity_factors, patience_options)
             if total_ops % l == 0]
    if measure is None:
        measure = _mix_measure(kind, capacity, total_ops, reps)
    return _search(key, cands, measure, cache_path, force)


def _arch_or(default: str, measure) -> str:
    return default if measure is not None else _device_arch()


def checksums(v: np.ndarray):
    """(count, wrapping sum of v, wrapping sum of v * v) of uint64 items."""
    with np.errstate(over="ignore"):
        return int(v.shape[0]), int(v.sum(dtype=np.uint64)), int((v * v).sum(dtype=np.uint64))


def _csum_add(a, b):
    m = (1 << 64) - 1
    return a[0] + b[0], (a[1] + b[1]) & m, (a[2] + b[2]) & m


def _mix_measure(kind, capacity, total_ops, reps):
    import torch

    from . import GQ_OK, Queue

    def run(c):
        ring = capacity * c.get("capacity_factor", 1)
        q = Queue(kind, ring, item_width=8, max_threads=c["lanes"], slot_mode=c["slot_mode"],
                  ticket_group=c["ticket_group"], patience=c["patience"],
                  ymc_pool_cells=(total_ops * (reps + 1) + ring) if kind == "ymc" else 0)
        try:
            pre = torch.arange(1, capacity // 2 + 1, dtype=torch.int64, device="cuda")
            q.enqueue_batch(pre)
            counts = torch.zeros(8, dtype=torch.int64, device="cuda")
            seed = [0]

            def launch():
                seed[0] += 1
                q.run_mix(seed[0], c["lanes"], total_ops // c["lanes"], counts)

            ms = _time_ms(torch, launch, reps)
            cnt = counts.cpu().numpy().view(np.uint64).tolist()
            err = q.check_error()
            if err != 0:
                raise RuntimeError(f"device error {err}")
            # conservation over all launches: prefill + enqueued = dequeued + left
            out = torch.zeros(ring, dtype=torch.int64, device="cuda")
            st = torch.zeros(ring, dtype=torch.uint8, device="cuda")
            left = []
            while True:
                q.dequeue_batch(out, st)
                ok = st.cpu().numpy() == GQ_OK
                if not ok.any():
                    break
                left.append(out.cpu().numpy().view(np.uint64)[ok])
            left = np.concatenate(left) if left else np.zeros(0, dtype=np.uint64)
            put = _csum_add(checksums(pre.cpu().numpy().view(np.uint64)), (cnt[0], cnt[6], cnt[7]))
            got = _csum_add((cnt[1], cnt[4], cnt[5]), checksums(left))
            if put != got:
                raise RuntimeError(f"items not conserved: in {put}, out {got}")
            return ms, (cnt[0] + cnt[1]) / (reps + 1)
        finally:
            q.close()

    return run


def tune_multi(kind: str, capacities, waves_per_256_slots=(0.5, 1, 2, 4), ops_factor: int = 4,
               reps: int = 3, cache_path: str = "", force: bool = False,
               measure: Callable[[Dict], tuple] = None) -> TuneResult:
    """Fastest lane allotment for the many-queue launch over queues of the
    given capacities, each doing ops_factor * n operations per step."""
    caps = [int(c) for c in capacities]
    sig = f"{len(caps)}q-{min(caps)}-{max(caps)}-{sum(caps)}"
    key = f"multi/{_arch_or('any', measure)}/{kind}/{sig}/x{ops_factor}"
    cands = [dict(waves_per_256_slots=w) for w in waves_per_256_slots]
    if measure is None:
        measure = _multi_measure(kind, caps, ops_factor, reps)
    return _search(key, cands, measure, cache_path, force)


def multi_lanes(caps, waves_per_256_slots: float, ops_factor: int):
    """Lanes per queue and the common operations per lane for an allotment:
    each queue gets max(1, round(w * n / 256)) wavefronts, the per-lane count
    is set so that the largest queue does ops_factor * n operations."""
    lanes = [64 * max(1, int(round(waves_per_256_slots * c / 256))) for c in caps]
    big = int(np.argmax(caps))
    ops = max(1, ops_factor * caps[big] // lanes[big])
    pad = (-sum(lanes)) % 256
    lanes[big] += pad
    return lanes, ops


def _multi_measure(kind, caps, ops_factor, reps):
    import torch

    from . import Multi, Queue

    def run(c):
        lanes, ops = multi_lanes(caps, c["waves_per_256_slots"], ops_factor)
        qs = [Queue(kind, n, item_width=8, max_threads=l,
                    ymc_pool_cells=(ops * l * (reps + 2) + n) if kind == "ymc" else 0)
              for n, l in zip(caps, lanes)]
        m = None
        try:
            for q, n in zip(qs, caps):
                q.enqueue_batch(torch.arange(1, n // 2 + 1, dtype=torch.int64, device="cuda"))
            m = Multi(qs, lanes, block=256)
            counts = torch.zeros(8 * len(qs), dtype=torch.int64, device="cuda")
            seed = [0]

            def launch():
                seed[0] += 1
                m.run_mix(seed[0], ops, counts)

            ms = _time_ms(torch, launch, reps)
            cnt = counts.cpu().numpy().reshape(-1, 8)
            return ms, float(cnt[:, 0].sum() + cnt[:, 1].sum()) / (reps + 1)
        finally:
            if m is not None:
                m.close()
            for q in qs:
                q.close()

    return run


def tune_prodcons(kind: str = "wfq", capacity: int = 1 << 16, waves: int = 1024,
                  prod_waves: int = 128, log2_inv_p: int = 0, items: int = 1 << 23,
                  patience_options=((16, 64), (64, 256), (256, 1024)),
                  help_delays=(16, 64, 256), time_limit_ms: int = 20000,
                  cache_path: str = "", force: bool = False,
                  measure: Callable[[Dict], tuple] = None) -> TuneResult:
    """Fastest (patience, help delay) for one imbalanced producer/consumer
    configuration: `waves` wavefronts of which the seed makes `prod_waves`
    producers, activity probability 2^-log2_inv_p, `items` items.  The
    measure returns (ms, successful operations); a run that does not finish
    or breaks conservation raises and is recorded as failed."""
    key = (f"prodcons/{_arch_or('any', measure)}/{kind}/cap{capacity}/w{waves}/p{prod_waves}"
           f"/a{log2_inv_p}/i{items}")
    cands = [dict(patience=list(pt), help_delay=d)
             for pt, d in itertools.product(patience_options, help_delays)]
    if measure is None:
        measure = _prodcons_measure(kind, capacity, waves, prod_waves, log2_inv_p, items,
                                    time_limit_ms)
    return _search(key, cands, measure, cache_path, force)


def _prodcons_measure(kind, capacity, waves, prod_waves, log2_inv_p, items, time_limit_ms):
    import torch

    import workloads

    from . import GQ_OK, Queue

    lanes = waves * 64

    def run(c):
        q = Queue(kind, capacity, item_width=8, max_threads=lanes,
                  patience=tuple(c["patience"]), help_delay=c["help_delay"])
        try:
            seed = workloads.run_seed(3, prod_waves + log2_inv_p)
            mask = workloads.producer_waves(seed, waves, prod_waves)
            role = torch.tensor(np.repeat(np.where(mask, 0, 1), 64).astype(np.uint8),
                                device="cuda")
            quota = -(-items // (prod_waves * 64))
            target = quota * prod_waves * 64
            counts = torch.zeros(8, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            q.run_prodcons(seed, lanes, 256, role, quota, target, log2_inv_p, 0, counts,
                           max_rounds=1 << 30, time_limit_ms=time_limit_ms)
            e1.record()
            torch.cuda.synchronize()
            c8 = counts.cpu().numpy().view(np.uint64)
            err = q.check_error()
            if err != GQ_OK or c8[0] != target or c8[1] != target or c8[4] != c8[6] \
                    or c8[5] != c8[7]:
                raise RuntimeError(f"run did not complete: error {err}, "
                                   f"{int(c8[0])}/{int(c8[1])} of {target}")
            return e0.elapsed_time(e1), 2 * target
        finally:
            q.close()

    return run
