"""ctypes binding of libgq.so (include/gq.h, include/gq_bench.h).

Argument marshalling only: every queue operation runs in the HIP kernels of
libgq.so.  PyTorch provides device memory (``torch.empty(..., device="cuda")``)
and the current HIP stream; nothing else.  There is no CPU fallback: if the
library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgq.so")

GQ_OK, GQ_EMPTY, GQ_FULL = 0, 1, 2
GQ_ERR_INVALID, GQ_ERR_NOMEM, GQ_ERR_HIP, GQ_ERR_RESIDENCY = -1, -2, -3, -4
GQ_ERR_CYCLE_BOUND, GQ_ERR_POOL_EXHAUSTED, GQ_ERR_DEVICE, GQ_ERR_TOO_LARGE = -5, -6, -7, -8

KINDS = {"lfq": 0, "wfq": 1, "ymc": 2}
SLOT_MODES = {"remap": 0, "padded": 1, "linear": 2}

# Every symbol the headers under include/ declare.
EXPORTS = (
    "gq_required_bytes", "gq_create", "gq_destroy", "gq_reset", "gq_enqueue_batch",
    "gq_dequeue_batch", "gq_device_view", "gq_read_stats", "gq_clear_stats",
    "gq_check_error", "gq_status_str", "gq_run_mix", "gq_run_balanced", "gq_run_prodcons",
    "gq_run_script", "gq_probe_faa", "gq_probe_cas", "gq_probe_copy", "gq_probe_fence",
    "gq_resident_blocks", "gq_device_info", "gq_multi_create", "gq_multi_run_mix",
    "gq_multi_capture", "gq_multi_replay", "gq_multi_destroy", "gq_bfs", "gq_bfs_ctl_bytes",
    "gq_bfs_static",
    "gq_serve_create", "gq_serve_run", "gq_serve_job_bytes", "gq_serve_destroy",
    "gq_run_timed", "gq_rt_create", "gq_rt_render", "gq_rt_check_error", "gq_rt_destroy",
)


class GQError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


GQ_OPT_FENCED = 1
GQ_OPT_WFQ_TUNING = 2


class _Options(ctypes.Structure):
    _fields_ = [("slot_mode", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("ymc_pool_cells", ctypes.c_uint64), ("wfq_patience_enq", ctypes.c_uint32),
                ("wfq_patience_deq", ctypes.c_uint32), ("wfq_help_delay", ctypes.c_uint32),
                ("ticket_group", ctypes.c_uint32)]


def make_options(slot_mode="linear", fenced=False, ymc_pool_cells=0, patience=None,
                 help_delay=None, ticket_group=0) -> _Options:
    flags = GQ_OPT_FENCED if fenced else 0
    pe, pd, hd = 64, 256, 64
    if patience is not None or help_delay is not None:
        flags |= GQ_OPT_WFQ_TUNING
        if patience is not None:
            pe, pd = (patience, patience) if isinstance(patience, int) else patience
        if help_delay is not None:
            hd = help_delay
    return _Options(SLOT_MODES[slot_mode], flags, ymc_pool_cells, pe, pd, hd, ticket_group)


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("ok_enq", "ok_deq", "full", "empty", "cas_fail", "tickets", "slow_enter",
                 "helps", "scans", "dropped")]


class _History(ctypes.Structure):
    _fields_ = [("val", ctypes.c_void_p), ("call", ctypes.c_void_p), ("ret", ctypes.c_void_p),
                ("opst", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("per_lane", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _RingView(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_void_p), ("head", ctypes.c_void_p), ("tail", ctypes.c_void_p),
                ("threshold", ctypes.c_void_p), ("records", ctypes.c_void_p),
                ("owner", ctypes.c_void_p),
                ("hint", ctypes.c_void_p), ("announce", ctypes.c_void_p)]


class _DevView(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("item_width", ctypes.c_uint32),
                ("log2_cap", ctypes.c_uint32), ("slot_mode", ctypes.c_uint32),
                ("max_threads", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("capacity", ctypes.c_uint64), ("data", ctypes.c_void_p),
                ("aq", _RingView), ("fq", _RingView), ("err", ctypes.c_void_p),
                ("stats", ctypes.c_void_p), ("ymc_cells", ctypes.c_void_p),
                ("ymc_pool_cells", ctypes.c_uint64), ("ymc_ctr", ctypes.c_void_p),
                ("ymc_handles", ctypes.c_void_p), ("patience_enq", ctypes.c_uint32),
                ("patience_deq", ctypes.c_uint32), ("help_delay", ctypes.c_uint32),
                ("group_lanes", ctypes.c_uint32), ("help_ctr", ctypes.c_void_p),
                ("ymc_hint", ctypes.c_void_p)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libgq.so not built at {path}; run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime.  Load it first so that libgq.so binds
    # to that same runtime (its libamdhip64.so.7 dependency then resolves to
    # the already-loaded copy); two runtimes in one process do not share
    # devices, memory or streams.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "gq_required_bytes": [I32, U64, U32, U32, P, P],
        "gq_create": [I32, U64, U32, U32, P, P, U64, P],
        "gq_destroy": [P],
        "gq_reset": [P, P],
        "gq_enqueue_batch": [P, P, U64, P, P, P],
        "gq_dequeue_batch": [P, P, U64, P, P, P],
        "gq_device_view": [P, P],
        "gq_read_stats": [P, P, P],
        "gq_clear_stats": [P, P],
        "gq_check_error": [P, P],
        "gq_run_mix": [P, U64, U32, U32, P, P, P, P],
        "gq_run_balanced": [P, U32, U32, P, P, P],
        "gq_run_prodcons": [P, U64, U32, U32, P, U32, U64, U32, U32, U32, U64, U32, P, P, P],
        "gq_run_script": [P, U32, U32, P, P, P, P, U32, P, P],
        "gq_probe_faa": [P, U32, U32, U32, U32, U32, P],
        "gq_probe_cas": [P, U64, U32, U32, U32, P],
        "gq_probe_copy": [P, P, U64, P],
        "gq_probe_fence": [P, U32, U32, U32, P],
        "gq_resident_blocks": [ctypes.c_char_p, I32, U32, P],
        "gq_device_info": [P, P, P, U32],
        "gq_multi_create": [U32, P, P, U32, P],
        "gq_multi_run_mix": [P, U64, U32, P, P, P],
        "gq_multi_capture": [P, U64, U32, P, P, P],
        "gq_multi_replay": [P, P],
        "gq_multi_destroy": [P],
        "gq_bfs": [P, P, P, P, U32, U32, P, U32, U32, P, U64, P],
        "gq_serve_create": [U32, U32, I32, U64, U32, U32, P],
        "gq_run_timed": [P, U32, U32, U32, U32, U32, P, P, P, P, P],
        "gq_serve_run": [P, U32, P, P, U32, P],
        "gq_serve_job_bytes": [P, U32, U64, P],
        "gq_serve_destroy": [P],
        "gq_rt_create": [I32, U32, U32, U32, U32, P],
        "gq_rt_render": [P, P, U32, P, P, P, P],
        "gq_rt_check_error": [P, P],
        "gq_rt_destroy": [P],
    }
    L.gq_bfs_ctl_bytes.restype = U64
    L.gq_bfs_ctl_bytes.argtypes = [U64]
    L.gq_bfs_static.restype = I32
    L.gq_bfs_static.argtypes = [I32, P, P, U32, U32, P, U32, U32, P, P]
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.gq_status_str.argtypes = [ctypes.c_int]
    L.gq_status_str.restype = ctypes.c_char_p
    return L


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def status_str(s: int) -> str:
    return lib().gq_status_str(int(s)).decode()


def _check(rc: int, what: str):
    if rc != GQ_OK:
        raise GQError(rc, what)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the queues run on the GPU only; no HIP device is visible")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_words(counts, words: int, what: str):
    """Device buffers are plain pointers at the C ABI: check their size here."""
    if counts.numel() * counts.element_size() < 8 * words:
        raise ValueError(f"{what} needs a counts buffer of at least {words} int64 words")


def _need_hist(hist, lanes: int, what: str):
    if hist is not None and hist.lanes < lanes:
        raise ValueError(f"{what}: history holds {hist.lanes} lanes, run uses {lanes}")


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def required_bytes(kind: str, capacity: int, item_width: int = 8, max_threads: int = 1,
                   slot_mode: str = "linear", ymc_pool_cells: int = 0, **opts) -> int:
    o = make_options(slot_mode, ymc_pool_cells=ymc_pool_cells, **opts)
    out = ctypes.c_uint64(0)
    _check(lib().gq_required_bytes(KINDS[kind], capacity, item_width, max_threads,
                                   ctypes.byref(o), ctypes.byref(out)), "gq_required_bytes")
    return int(out.value)


@dataclass
class Stats:
    ok_enq: int
    ok_deq: int
    full: int
    empty: int
    cas_fail: int
    tickets: int
    slow_enter: int
    helps: int
    scans: int
    dropped: int


class History:
    """Device history buffers for `lanes` lanes x `per_lane` records."""

    def __init__(self, lanes: int, per_lane: int):
        torch = _torch()
        n = lanes * per_lane
        self.lanes, self.per_lane = lanes, per_lane
        self.val = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.call = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.ret = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.opst = torch.zeros(n, dtype=torch.uint8, device="cuda")
        self.count = torch.zeros(lanes, dtype=torch.int32, device="cuda")

    def c(self) -> _History:
        return _History(self.val.data_ptr(), self.call.data_ptr(), self.ret.data_ptr(),
                        self.opst.data_ptr(), self.count.data_ptr(), self.per_lane, 0)

    def to_numpy(self):
        """Returns (proc, op, st, val, call, ret, overflow) for the stored records,
        grouped by lane in program order; overflow = lanes that executed more
        operations than were stored."""
        cnt = self.count.cpu().numpy().astype(np.int64)
        stored = np.minimum(cnt, self.per_lane)
        lane_start = np.repeat(np.arange(self.lanes, dtype=np.int64) * self.per_lane, stored)
        within = np.arange(int(stored.sum()), dtype=np.int64) - \
            np.repeat(np.cumsum(stored) - stored, stored)
        idx = lane_start + within
        proc = np.repeat(np.arange(self.lanes, dtype=np.uint32), stored)
        opst = self.opst.cpu().numpy()[idx]
        val = self.val.cpu().numpy().view(np.uint64)[idx]
        call = self.call.cpu().numpy().view(np.uint64)[idx]
        ret = self.ret.cpu().numpy().view(np.uint64)[idx]
        return proc, (opst & 1).astype(np.uint8), (opst >> 1).astype(np.uint8), val, call, ret, \
            int((cnt > self.per_lane).sum())


class Queue:
    """One device queue.  kind: 'lfq' | 'wfq' | 'ymc'."""

    def __init__(self, kind: str, capacity: int, item_width: int = 8, max_threads: int = 1,
                 slot_mode: str = "linear", ymc_pool_cells: int = 0, fenced: bool = False,
                 patience=None, help_delay=None, ticket_group: int = 0):
        torch = _torch()
        self.kind, self.capacity, self.item_width = kind, capacity, item_width
        self.max_threads = max_threads
        self._opts = make_options(slot_mode, fenced, ymc_pool_cells, patience, help_delay,
                                  ticket_group)
        o = self._opts
        out = ctypes.c_uint64(0)
        _check(lib().gq_required_bytes(KINDS[kind], capacity, item_width, max_threads,
                                       ctypes.byref(o), ctypes.byref(out)), "gq_required_bytes")
        nbytes = int(out.value)
        # torch owns the memory; 256-byte alignment comes from the caching allocator
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p(0)
        _check(lib().gq_create(KINDS[kind], capacity, item_width, max_threads,
                               ctypes.byref(self._opts), _ptr(self._buf), nbytes,
                               ctypes.byref(h)), "gq_create")
        self._h = h
        self.nbytes = nbytes

    def close(self):
        if getattr(self, "_h", None):
            lib().gq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def reset(self, stream=None):
        _check(lib().gq_reset(self._h, _stream(stream)), "gq_reset")

    def enqueue_batch(self, items, status=None, num_ok=None, stream=None):
        _check(lib().gq_enqueue_batch(self._h, _ptr(items), items.numel(), _ptr(status),
                                      _ptr(num_ok), _stream(stream)), "gq_enqueue_batch")

    def dequeue_batch(self, out, status=None, num_ok=None, stream=None):
        _check(lib().gq_dequeue_batch(self._h, _ptr(out), out.numel(), _ptr(status),
                                      _ptr(num_ok), _stream(stream)), "gq_dequeue_batch")

    def device_view(self) -> _DevView:
        v = _DevView()
        _check(lib().gq_device_view(self._h, ctypes.byref(v)), "gq_device_view")
        return v

    def stats(self, stream=None) -> Stats:
        s = _Stats()
        _check(lib().gq_read_stats(self._h, ctypes.byref(s), _stream(stream)), "gq_read_stats")
        return Stats(*[getattr(s, f[0]) for f in _Stats._fields_])

    def clear_stats(self, stream=None):
        _check(lib().gq_clear_stats(self._h, _stream(stream)), "gq_clear_stats")

    def check_error(self, stream=None) -> int:
        return int(lib().gq_check_error(self._h, _stream(stream)))

    # ---- workload drivers --------------------------------------------------
    def run_mix(self, seed: int, lanes: int, ops_per_lane: int, counts, hist: History = None,
                stream=None, lane_enq=None):
        """Mixed 50/50 workload.  counts: 8 int64 words, added to: {ok_enq,
        ok_deq, full, empty, S1_deq, S2_deq, S1_enq, S2_enq} (wrapping sums of
        v and v*v).  lane_enq (optional int32[lanes]): each lane's count of
        successful enqueues."""
        _need_words(counts, 8, "run_mix")
        _need_hist(hist, lanes, "run_mix")
        if lane_enq is not None and lane_enq.numel() * lane_enq.element_size() < 4 * lanes:
            raise ValueError("run_mix: lane_enq needs one 32-bit word per lane")
        hc = hist.c() if hist is not None else None
        _check(lib().gq_run_mix(self._h, seed, lanes, ops_per_lane, _ptr(counts), _ptr(lane_enq),
                                ctypes.byref(hc) if hc is not None else None, _stream(stream)),
               "gq_run_mix")

    def run_balanced(self, lanes: int, rounds: int, counts, hist: History = None, stream=None):
        _need_words(counts, 4, "run_balanced")
        _need_hist(hist, lanes, "run_balanced")
        hc = hist.c() if hist is not None else None
        _check(lib().gq_run_balanced(self._h, lanes, rounds, _ptr(counts),
                                     ctypes.byref(hc) if hc is not None else None,
                                     _stream(stream)), "gq_run_balanced")

    def run_prodcons(self, seed: int, lanes: int, block: int, lane_role, items_per_producer: int,
                     target: int, log2_inv_p: int, token_mode: int, counts, hist: History = None,
                     jitter: int = 0, max_rounds: int = 1 << 26, time_limit_ms: int = 60000,
                     stream=None):
        _need_words(counts, 8, "run_prodcons")
        _need_hist(hist, lanes, "run_prodcons")
        if lane_role.numel() < lanes:
            raise ValueError("lane_role must hold one entry per lane")
        hc = hist.c() if hist is not None else None
        _check(lib().gq_run_prodcons(self._h, seed, lanes, block, _ptr(lane_role),
                                     items_per_producer, target, log2_inv_p, token_mode, jitter,
                                     max_rounds, time_limit_ms, _ptr(counts),
                                     ctypes.byref(hc) if hc is not None else None,
                                     _stream(stream)), "gq_run_prodcons")

    def run_timed(self, mode: str, lanes: int, counts, ctl, prod_pct: int = 50,
                  warmup_us: int = 1000, window_us: int = 5000, lane_enq=None,
                  hist: History = None, stream=None):
        """Fixed-duration run; mode 'balanced' or 'split'.  counts: 10 int64
        words (added to; see gq_run_timed); ctl: at least one int64 word of
        scratch; lane_enq: optional int32 per lane; hist: optional History."""
        _need_words(counts, 10, "run_timed")
        _need_words(ctl, 1, "run_timed ctl")
        if lane_enq is not None and lane_enq.numel() * lane_enq.element_size() < 4 * lanes:
            raise ValueError("run_timed: lane_enq needs one int32 per lane")
        _need_hist(hist, lanes, "run_timed")
        hc = hist.c() if hist is not None else None
        _check(lib().gq_run_timed(self._h, {"balanced": 0, "split": 1}[mode], lanes, prod_pct,
                                  warmup_us, window_us, _ptr(counts), _ptr(ctl),
                                  _ptr(lane_enq) if lane_enq is not None else None,
                                  ctypes.byref(hc) if hc is not None else None,
                                  _stream(stream)), "gq_run_timed")

    def run_script(self, lanes: int, spread: bool, ops, args, pauses, n_ops, max_ops: int,
                   hist: History, stream=None):
        hc = hist.c()
        _check(lib().gq_run_script(self._h, lanes, 1 if spread else 0, _ptr(ops), _ptr(args),
                                   _ptr(pauses), _ptr(n_ops), max_ops, ctypes.byref(hc),
                                   _stream(stream)), "gq_run_script")


# ---- probes and device info ---------------------------------------------------
def probe_faa(ctr, lanes: int, iters: int, per_lane: bool, ncounters: int = 1,
              spacing_bytes: int = 256, stream=None):
    assert ctr.numel() * ctr.element_size() >= ncounters * spacing_bytes
    _check(lib().gq_probe_faa(_ptr(ctr), lanes, iters, 1 if per_lane else 0, ncounters,
                              spacing_bytes, _stream(stream)), "gq_probe_faa")


def probe_cas(slots, nslots: int, stride_bytes: int, lanes: int, iters: int, stream=None):
    _check(lib().gq_probe_cas(_ptr(slots), nslots, stride_bytes, lanes, iters, _stream(stream)),
           "gq_probe_cas")


def probe_copy(dst, src, n: int, stream=None):
    _check(lib().gq_probe_copy(_ptr(dst), _ptr(src), n, _stream(stream)), "gq_probe_copy")


def probe_fence(lines, lanes: int, iters: int, mode: int, stream=None):
    _check(lib().gq_probe_fence(_ptr(lines), lanes, iters, mode, _stream(stream)),
           "gq_probe_fence")


def resident_blocks(kernel: str, kind: str, block: int) -> int:
    out = ctypes.c_uint32(0)
    _check(lib().gq_resident_blocks(kernel.encode(), KINDS[kind], block, ctypes.byref(out)),
           "gq_resident_blocks")
    return int(out.value)


def device_info():
    cus, wave = ctypes.c_uint32(0), ctypes.c_uint32(0)
    name = ctypes.create_string_buffer(64)
    _check(lib().gq_device_info(ctypes.byref(cus), ctypes.byref(wave), name, 64), "gq_device_info")
    return {"cus": int(cus.value), "wave": int(wave.value), "arch": name.value.decode()}


class Multi:
    """Many independent queues driven by one kernel launch (and a hipGraph)."""

    def __init__(self, queues, lanes_per_queue, block: int = 256):
        self.queues = list(queues)
        self.lanes = [int(x) for x in lanes_per_queue]
        arr = (ctypes.c_void_p * len(self.queues))(*[q.handle for q in self.queues])
        lp = (ctypes.c_uint32 * len(self.lanes))(*self.lanes)
        h = ctypes.c_void_p(0)
        _check(lib().gq_multi_create(len(self.queues), arr, lp, block, ctypes.byref(h)),
               "gq_multi_create")
        self._h = h

    def run_mix(self, seed: int, ops_per_lane: int, counts, hist: History = None, stream=None):
        _need_words(counts, 8 * len(self.queues), "Multi.run_mix")
        _need_hist(hist, sum(self.lanes), "Multi.run_mix")
        hc = hist.c() if hist is not None else None
        _check(lib().gq_multi_run_mix(self._h, seed, ops_per_lane, _ptr(counts),
                                      ctypes.byref(hc) if hc is not None else None,
                                      _stream(stream)), "gq_multi_run_mix")

    def capture(self, seed: int, ops_per_lane: int, counts, stream, hist: History = None):
        _need_words(counts, 8 * len(self.queues), "Multi.capture")
        _need_hist(hist, sum(self.lanes), "Multi.capture")
        hc = hist.c() if hist is not None else None
        self._hist_c = hc  # the graph keeps the history's device pointers
        _check(lib().gq_multi_capture(self._h, seed, ops_per_lane, _ptr(counts),
                                      ctypes.byref(hc) if hc is not None else None,
                                      _stream(stream)), "gq_multi_capture")

    def replay(self, stream):
        _check(lib().gq_multi_replay(self._h, _stream(stream)), "gq_multi_replay")

    def close(self):
        if getattr(self, "_h", None):
            lib().gq_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bfs_ctl_bytes(nnz: int) -> int:
    """Workspace bytes for bfs() on a graph of nnz adjacency entries."""
    return int(lib().gq_bfs_ctl_bytes(nnz))


def bfs(qa: Queue, qb: Queue, offsets, cols, root: int, level, lanes: int, block: int, ctl,
        stream=None):
    """Launch the queue-driven BFS; offsets/cols/level/ctl are CUDA tensors
    (ctl: the workspace, at least 4 KiB; bfs_ctl_bytes(nnz) for the full hub
    list)."""
    nv = offsets.numel() - 1
    ctl_bytes = ctl.numel() * ctl.element_size()
    if level.numel() < nv or cols.numel() < 1 or ctl_bytes < 4096:
        raise ValueError("bfs: level must hold nv entries, ctl at least 4 KiB")
    _check(lib().gq_bfs(qa.handle, qb.handle, _ptr(offsets), _ptr(cols), offsets.numel() - 1,
                        root, _ptr(level), lanes, block, _ptr(ctl), ctl_bytes, _stream(stream)),
           "gq_bfs")


# ---------------------------------------------------------------------------
# Serving (include/gq_serve.h)
# ---------------------------------------------------------------------------
class _ServeRequest(ctypes.Structure):
    _fields_ = [("d_offsets", ctypes.c_void_p), ("d_cols", ctypes.c_void_p),
                ("d_levels_out", ctypes.c_void_p), ("nnz", ctypes.c_uint64),
                ("nv", ctypes.c_uint32), ("root", ctypes.c_uint32)]


class _ServeResult(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("device_ns", ctypes.c_int64),
                ("level_hash", ctypes.c_uint64), ("levels", ctypes.c_uint64),
                ("scanned", ctypes.c_uint64), ("job_bytes", ctypes.c_uint64),
                ("team", ctypes.c_uint32), ("status", ctypes.c_int32)]


SERVE_HASH_SEED = 0x5EED1E7E15


class Server:
    """A persistent serving kernel (gq_serve_create .. gq_serve_destroy).

    While it exists it occupies the GPU: do not call torch.cuda.synchronize()
    (a device-wide wait) until close(); put the graphs on the device first.
    Graph tensors passed to run() must stay alive until run() returns."""

    def __init__(self, teams: int, team_lanes: int = 1024, kind: str = "lfq",
                 budget_bytes: int = 16 << 30, ring_slots: int = 1024,
                 idle_timeout_ms: int = 0):
        h = ctypes.c_void_p(0)
        _check(lib().gq_serve_create(teams, team_lanes, KINDS[kind], budget_bytes, ring_slots,
                                     idle_timeout_ms, ctypes.byref(h)), "gq_serve_create")
        self._h = h
        self.teams, self.team_lanes, self.kind = teams, team_lanes, kind
        self.budget_bytes, self.ring_slots = budget_bytes, ring_slots

    def job_bytes(self, nv: int, nnz: int) -> int:
        out = ctypes.c_uint64(0)
        _check(lib().gq_serve_job_bytes(self._h, nv, nnz, ctypes.byref(out)),
               "gq_serve_job_bytes")
        return int(out.value)

    def run(self, requests, arrival_ns, max_inflight: int = None):
        """requests: sequence of (offsets, cols, root) or (offsets, cols, root,
        levels_out) with int32 CUDA tensors (levels_out: nv entries, receives
        the job's levels).  arrival_ns: non-decreasing schedule (ns from the
        call).  Returns a dict of numpy arrays, one entry per request."""
        n = len(requests)
        reqs = (_ServeRequest * max(1, n))()
        for i, rq in enumerate(requests):
            off, cols, root = rq[:3]
            out_t = rq[3] if len(rq) > 3 else None
            nv = off.numel() - 1
            if out_t is not None and out_t.numel() < nv:
                raise ValueError("levels_out must hold nv entries")
            reqs[i] = _ServeRequest(off.data_ptr(), cols.data_ptr(),
                                    out_t.data_ptr() if out_t is not None else None,
                                    cols.numel(), nv, int(root))
        arr = np.ascontiguousarray(np.asarray(arrival_ns, dtype=np.int64))
        if len(arr) != n:
            raise ValueError("one arrival time per request")
        res = (_ServeResult * max(1, n))()
        mi = self.ring_slots if max_inflight is None else max_inflight
        _check(lib().gq_serve_run(self._h, n, reqs, arr.ctypes.data, mi, res), "gq_serve_run")
        # explicit dtypes: 64-bit hashes above 2^63 must not pass through float
        dt = {ctypes.c_int64: np.int64, ctypes.c_uint64: np.uint64, ctypes.c_uint32: np.uint32,
              ctypes.c_int32: np.int32}
        return {name: np.array([getattr(res[i], name) for i in range(n)], dtype=dt[ct])
                for name, ct in _ServeResult._fields_}

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().gq_serve_destroy(h), "gq_serve_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- tile-based wavefront ray tracer (include/gq_rt.h) ----------------------
RT_QUEUES, RT_COMPACT = 0, 1
RT_MAX_SPHERES, RT_MAX_PLANES = 128, 8


class _RtScene(ctypes.Structure):
    _fields_ = [("spheres", ctypes.c_void_p), ("planes", ctypes.c_void_p),
                ("n_spheres", ctypes.c_uint32), ("n_planes", ctypes.c_uint32),
                ("camera", ctypes.c_float * 7), ("light", ctypes.c_float * 3),
                ("shade", ctypes.c_float * 2), ("background", ctypes.c_float * 3),
                ("max_bounces", ctypes.c_uint32)]


class RayTracer:
    """Per-tile queues of `kind` over a width x height image (gq_rt_create ..
    gq_rt_destroy).  ``render(scene)`` takes a scene dict of float32 arrays
    (the layout gq_rt.h documents) and returns (image [h*w, 3] float32,
    segments [h*w] int32, stats [4] int64) as device tensors."""

    def __init__(self, kind: str, width: int, height: int, tile: int = 32, lanes: int = 8192):
        self.width, self.height, self.kind = width, height, kind
        h = ctypes.c_void_p(0)
        _check(lib().gq_rt_create(KINDS[kind], width, height, tile, lanes, ctypes.byref(h)),
               "gq_rt_create")
        self._h = h
        self._scene_keep = None

    def close(self):
        if getattr(self, "_h", None):
            lib().gq_rt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scene(self, scene: dict):
        torch = _torch()
        sph = torch.as_tensor(scene["spheres"], dtype=torch.float32).reshape(-1).contiguous().cuda()
        pl = torch.as_tensor(scene["planes"], dtype=torch.float32).reshape(-1).contiguous().cuda()
        sc = _RtScene()
        sc.spheres = sph.data_ptr() if sph.numel() else None
        sc.planes = pl.data_ptr() if pl.numel() else None
        sc.n_spheres = len(scene["spheres"])
        sc.n_planes = len(scene["planes"])
        for name, n in (("camera", 7), ("light", 3), ("shade", 2), ("background", 3)):
            arr = getattr(sc, name)
            for i in range(n):
                arr[i] = float(scene[name][i])
        sc.max_bounces = int(scene["max_bounces"])
        self._scene_keep = (sph, pl)
        self._scene = sc

    def render(self, method: int = RT_QUEUES, image=None, segments=None, stats=None, stream=None):
        torch = _torch()
        n = self.width * self.height
        if image is None:
            image = torch.empty(n * 3, dtype=torch.float32, device="cuda")
        if segments is None:
            segments = torch.empty(n, dtype=torch.int32, device="cuda")
        if stats is None:
            stats = torch.zeros(4, dtype=torch.int64, device="cuda")
        if image.numel() < n * 3 or segments.numel() < n or stats.numel() < 4:
            raise ValueError("render: output buffers too small")
        _check(lib().gq_rt_render(self._h, ctypes.byref(self._scene), method, _ptr(image),
                                  _ptr(segments), _ptr(stats), _stream(stream)), "gq_rt_render")
        return image.view(n, 3), segments, stats

    def check_error(self, stream=None) -> int:
        return int(lib().gq_rt_check_error(self._h, _stream(stream)))
