"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no queue arithmetic.  It defines the workloads only: the
counter-based random stream, the per-operation roles and tokens, the wave
role split of the small producer/consumer run, and the BFS graphs.

Random stream.  ``splitmix64(seed, c)`` is the c-th output (counting from 0) of
the SplitMix64 generator seeded with ``seed`` (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014; Vigna's public
reference implementation): state_c = seed + (c + 1) * 0x9E3779B97F4A7C15, then
the finalizer z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31.  Because it is counter based, the GPU
kernels evaluate the same function on their own (their own implementation of
the same published definition) and never need the arrays built here.

Counter layout: c = (stream << 32) | k, where ``stream`` is the global lane id
(or a wave/graph id) and ``k`` the per-stream draw index.

Tokens follow the paper's device FIFO check (Section IV): a producer lane
``tid`` emits (tid << 32) | (seq + 1) for its seq-th successful enqueue.  The
small uint32 run uses (producer_id << 20) | seq instead (its payload is 32-bit).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_GG_SRC = os.path.join(_HERE, "graphgen.c")
_GG_LIB = os.path.join(_HERE, "libgraphgen.so")


def build() -> str:
    """Compile the C graph builders (gcc, always rebuilds)."""
    subprocess.run(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread", _GG_SRC, "-o",
                    _GG_LIB + ".tmp"], check=True)
    os.replace(_GG_LIB + ".tmp", _GG_LIB)
    return _GG_LIB


_gg = None


def _threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def _graphgen():
    global _gg
    if _gg is None:
        if not os.path.exists(_GG_LIB):
            build()
        L = ctypes.CDLL(_GG_LIB)
        P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.wl_rmat_pairs.argtypes = [U32, U64, U64, U64, U64, U64, P, P, U32, P]
        L.wl_rmat_pairs.restype = ctypes.c_int
        L.wl_csr.argtypes = [U64, U64, P, P, P, P]
        L.wl_csr.restype = ctypes.c_int64
        L.wl_csr_par.argtypes = [U64, U64, P, P, P, P, U32]
        L.wl_csr_par.restype = ctypes.c_int64
        _gg = L
    return _gg

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 20260601


def run_seed(config: int, run: int) -> int:
    """Per-run seed: base_seed + 1000 * config + run."""
    return BASE_SEED + 1000 * config + run


def splitmix64(seed, c):
    """c-th output of SplitMix64 seeded with ``seed`` (vectorised over c)."""
    with np.errstate(over="ignore"):
        c = np.asarray(c, dtype=np.uint64)
        z = np.uint64(seed) + (c + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
        return z ^ (z >> np.uint64(31))


def counter(stream, k):
    s = np.asarray(stream, dtype=np.uint64)
    kk = np.asarray(k, dtype=np.uint64)
    return (s << np.uint64(32)) | kk


# ----------------------------------------------------------------------------
# Mixed 50/50 throughput workload: each op of lane g, draw k, is an enqueue when
# the top bit of splitmix64(seed, (g << 32) | k) is 0, else a dequeue.
# ----------------------------------------------------------------------------
ROLE_ENQ = 0
ROLE_DEQ = 1


def mix_roles(seed: int, lanes: int, ops_per_lane: int, lane0: int = 0) -> np.ndarray:
    """uint8 array [lanes, ops_per_lane] of roles (0 = enqueue, 1 = dequeue)."""
    g = np.arange(lane0, lane0 + lanes, dtype=np.uint64)[:, None]
    k = np.arange(ops_per_lane, dtype=np.uint64)[None, :]
    r = splitmix64(seed, counter(g, k))
    return (r >> np.uint64(63)).astype(np.uint8)


def mix_tokens(roles: np.ndarray, lane0: int = 0) -> np.ndarray:
    """Token each op would enqueue if every enqueue succeeds in order.

    For lane g the j-th enqueue (0-based) carries (g << 32) | (j + 1).  For
    dequeue slots the entry is 0.  Only valid as a sequential replay input when
    enqueues never fail; the concurrent harness numbers successful enqueues.
    """
    lanes, ops = roles.shape
    is_enq = roles == ROLE_ENQ
    seq = np.cumsum(is_enq, axis=1, dtype=np.uint64)  # 1-based count
    g = np.arange(lane0, lane0 + lanes, dtype=np.uint64)[:, None]
    tok = (g << np.uint64(32)) | seq
    return np.where(is_enq, tok, np.uint64(0))


def token(tid, seq):
    """The paper's FIFO-conformance token (tid << 32) | (seq + 1)."""
    return (np.uint64(tid) << np.uint64(32)) | (np.uint64(seq) + np.uint64(1))


# ----------------------------------------------------------------------------
# Small producer/consumer run (uint32 payload (pid << 20) | seq): 16 waves, the
# seed picks which 8 are producers: the 8 waves with the smallest draws
# splitmix64(seed, w), ties broken by wave id.
# ----------------------------------------------------------------------------
def producer_waves(seed: int, n_waves: int = 16, n_prod: int = 8) -> np.ndarray:
    r = splitmix64(seed, np.arange(n_waves, dtype=np.uint64))
    order = np.lexsort((np.arange(n_waves), r))
    mask = np.zeros(n_waves, dtype=bool)
    mask[order[:n_prod]] = True
    return mask


def small_token(pid: int, seq: int) -> int:
    return (int(pid) << 20) | int(seq)


# ----------------------------------------------------------------------------
# Divergent-activity workload: lane g is active in round k iff
# splitmix64(seed, (g << 32) | k) >> (64 - j) == 0, for p = 2^-j (j = 0 always).
# ----------------------------------------------------------------------------
def active_draw(seed: int, lanes, rounds, log2_inv_p: int) -> np.ndarray:
    if log2_inv_p == 0:
        return np.ones(np.broadcast(np.asarray(lanes), np.asarray(rounds)).shape, dtype=bool)
    r = splitmix64(seed, counter(lanes, rounds))
    return (r >> np.uint64(64 - log2_inv_p)) == 0


# ----------------------------------------------------------------------------
# Graphs (CSR, undirected, uint32 offsets and columns).
# ----------------------------------------------------------------------------
def _csr_from_pairs(nv: int, src: np.ndarray, dst: np.ndarray):
    """Symmetrise, drop self loops, deduplicate, return (offsets, cols)."""
    src = src.astype(np.uint64)
    dst = dst.astype(np.uint64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique((a << np.uint64(32)) | b)
    rows = (key >> np.uint64(32)).astype(np.int64)
    cols = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    counts = np.bincount(rows, minlength=nv)
    offsets = np.zeros(nv + 1, dtype=np.uint64)
    np.cumsum(counts, out=offsets[1:])
    if offsets[-1] >= 2**32:
        raise ValueError("graph too large for uint32 offsets")
    return offsets.astype(np.uint32), cols


def _csr_fast(nv: int, src: np.ndarray, dst: np.ndarray):
    src = np.ascontiguousarray(src, dtype=np.uint64)
    dst = np.ascontiguousarray(dst, dtype=np.uint64)
    off = np.zeros(nv + 1, dtype=np.uint32)
    cols = np.zeros(2 * len(src) + 1, dtype=np.uint32)
    nnz = _graphgen().wl_csr_par(nv, len(src), src.ctypes.data, dst.ctypes.data,
                                 off.ctypes.data, cols.ctypes.data, _threads())
    if nnz < 0:
        raise ValueError("graph too large for uint32 offsets")
    return off, cols[:nnz].copy()


def rmat_graph(scale: int, edgefactor: int = 16, a=0.57, b=0.19, c=0.19,
               seed: int = BASE_SEED, permute: bool = True, fast: bool = True):
    """Graph500-style R-MAT graph (no noise), seeded vertex permutation.

    Edge e, level l: the quadrant is chosen by u = splitmix64(seed,
    (e << 8) | l) / 2^64 against the cumulative probabilities a, a+b, a+b+c.
    Then symmetrised, self loops dropped, duplicates removed.  fast=True uses
    the C builders (identical output), fast=False the numpy definition below.
    """
    nv = 1 << scale
    ne = edgefactor * nv
    ta = np.uint64(int(a * 2**64) - 1)
    tab = np.uint64(int((a + b) * 2**64) - 1)
    tabc = np.uint64(int((a + b + c) * 2**64) - 1)
    if fast:
        src = np.zeros(ne, dtype=np.uint64)
        dst = np.zeros(ne, dtype=np.uint64)
        perm = np.ascontiguousarray(_rmat_perm(nv, seed)) if permute else None
        _graphgen().wl_rmat_pairs(scale, ne, int(seed) & (2**64 - 1), int(ta), int(tab), int(tabc),
                                  src.ctypes.data, dst.ctypes.data, _threads(),
                                  perm.ctypes.data if perm is not None else None)
        return _csr_fast(nv, src, dst)
    e = np.arange(ne, dtype=np.uint64)
    src = np.zeros(ne, dtype=np.uint64)
    dst = np.zeros(ne, dtype=np.uint64)
    for lvl in range(scale):
        u = splitmix64(seed, (e << np.uint64(8)) | np.uint64(lvl))
        right = ((u >= ta) & (u < tab)) | (u >= tabc)   # quadrants b, d
        down = u >= tab                                  # quadrants c, d
        bit = np.uint64(1 << (scale - 1 - lvl))
        src |= np.where(down, bit, np.uint64(0))
        dst |= np.where(right, bit, np.uint64(0))
    if permute:
        perm = _rmat_perm(nv, seed)
        src = perm[src.astype(np.int64)]
        dst = perm[dst.astype(np.int64)]
    return _csr_from_pairs(nv, src, dst)


def _rmat_perm(nv: int, seed: int) -> np.ndarray:
    """Seeded vertex relabelling: vertex v becomes the rank of its draw."""
    return np.argsort(splitmix64(seed ^ 0x5DEECE66D, np.arange(nv, dtype=np.uint64)),
                      kind="stable").astype(np.uint64)


def grid_graph(rows: int, cols: int, fast: bool = True):
    """rows x cols 4-neighbour grid, vertex id r * cols + c."""
    nv = rows * cols
    v = np.arange(nv, dtype=np.uint64).reshape(rows, cols)
    right = (v[:, :-1].ravel(), v[:, 1:].ravel())
    down = (v[:-1, :].ravel(), v[1:, :].ravel())
    src = np.concatenate([right[0], down[0]])
    dst = np.concatenate([right[1], down[1]])
    return _csr_fast(nv, src, dst) if fast else _csr_from_pairs(nv, src, dst)


def bfs_root(offsets: np.ndarray, seed: int) -> int:
    """Seeded uniform root among vertices of positive degree."""
    deg = np.diff(offsets.astype(np.int64))
    cand = np.nonzero(deg > 0)[0]
    if len(cand) == 0:
        return 0
    r = int(splitmix64(seed, np.uint64(0xB0F5)))
    return int(cand[r % len(cand)])
