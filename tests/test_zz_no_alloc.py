"""The allocation-free BFS entry point (gq_bfs_static), called through the C
ABI: its levels must equal those of gq_bfs (caller-created queues and
workspace) and the CPU BFS (O7), bit for bit, on two calls in a row -- the
second on a smaller graph, so stale contents of the shared static array from
the first call would show -- for both bounded queue kinds."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import torch

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def run_static(kind, off, cols, root, lanes, block=256):
    import paper_2606_01693_amd as gq
    T = torch()
    nv = len(off) - 1
    d_off = T.tensor(off.astype(np.int32), device="cuda")
    d_cols = T.tensor(cols.astype(np.int32), device="cuda")
    level = T.full((nv,), 7, dtype=T.int32, device="cuda")
    info = T.full((4,), -1, dtype=T.int64, device="cuda")
    rc = gq.lib().gq_bfs_static(gq.KINDS[kind], _ptr(d_off), _ptr(d_cols), nv, root,
                                _ptr(level), lanes, block, _ptr(info), None)
    assert rc == gq.GQ_OK, gq.status_str(rc)
    T.cuda.synchronize()
    return level.cpu().numpy().view(np.uint32), info.cpu().numpy()


def run_queues(kind, off, cols, root, lanes, block=256):
    import paper_2606_01693_amd as gq
    T = torch()
    nv = len(off) - 1
    cap = 64
    while cap < nv:
        cap *= 2
    qa = gq.Queue(kind, cap, item_width=4, max_threads=lanes)
    qb = gq.Queue(kind, cap, item_width=4, max_threads=lanes)
    d_off = T.tensor(off.astype(np.int32), device="cuda")
    d_cols = T.tensor(cols.astype(np.int32), device="cuda")
    level = T.empty(nv, dtype=T.int32, device="cuda")
    ctl = T.zeros(gq.bfs_ctl_bytes(len(cols)) // 8, dtype=T.int64, device="cuda")
    gq.bfs(qa, qb, d_off, d_cols, root, level, lanes, block, ctl)
    T.cuda.synchronize()
    assert qa.check_error() == gq.GQ_OK and qb.check_error() == gq.GQ_OK
    out = level.cpu().numpy().view(np.uint32)
    qa.close()
    qb.close()
    return out


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
def test_static_bfs_equals_queue_bfs(kind):
    # first call: R-MAT scale 18 (the maximum vertex count), hubs included;
    # second call: a 100 x 100 grid, far smaller
    big = workloads.rmat_graph(18, 16, seed=31)
    small = workloads.grid_graph(100, 100)
    cases = [(big, workloads.bfs_root(big[0], 31), 8192), (small, 4321, 2048)]
    for (off, cols), root, lanes in cases:
        print(f"[case] static bfs kind={kind} nv={len(off) - 1} m={len(cols)} root={root} "
              f"lanes={lanes}", flush=True)
        exp, nl, scanned = oracle.bfs(off, cols, root)
        got, info = run_static(kind, off, cols, root, lanes)
        ref = run_queues(kind, off, cols, root, lanes)
        assert np.array_equal(ref, exp)
        assert np.array_equal(got, ref)
        assert info[0] == 0
        assert info[1] in (nl, nl + 1)
        assert info[2] == scanned


def test_static_bfs_refuses_too_large():
    import paper_2606_01693_amd as gq
    T = torch()
    z = T.zeros(4, dtype=T.int32, device="cuda")
    rc = gq.lib().gq_bfs_static(gq.KINDS["lfq"], _ptr(z), _ptr(z), (1 << 18) + 1, 0, _ptr(z),
                                256, 256, None, None)
    assert rc == gq.GQ_ERR_TOO_LARGE
    rc = gq.lib().gq_bfs_static(gq.KINDS["lfq"], _ptr(z), _ptr(z), 3, 0, _ptr(z), 16384, 256,
                                None, None)
    assert rc == gq.GQ_ERR_TOO_LARGE
