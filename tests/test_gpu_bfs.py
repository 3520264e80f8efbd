"""Queue-driven BFS on the GPU: levels must equal the CPU BFS (oracle O7)
bit-exactly, on small graphs and on the full-size R-MAT (scale 22) and
4096 x 4096 grid inputs."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import torch

pytestmark = pytest.mark.gpu


def run_bfs(kind, off, cols, root, lanes, block=256, ymc_cells=0):
    import paper_2606_01693_amd as gq
    T = torch()
    nv = len(off) - 1
    cap = 1 << max(1, int(np.ceil(np.log2(max(nv, 2)))))
    qa = gq.Queue(kind, cap, item_width=4, max_threads=lanes, ymc_pool_cells=ymc_cells)
    qb = gq.Queue(kind, cap, item_width=4, max_threads=lanes, ymc_pool_cells=ymc_cells)
    d_off = T.tensor(off.astype(np.int32), device="cuda")
    d_cols = T.tensor(cols.astype(np.int32), device="cuda") if len(cols) else \
        T.zeros(1, dtype=T.int32, device="cuda")
    level = T.empty(nv, dtype=T.int32, device="cuda")
    ctl = T.zeros(512, dtype=T.int64, device="cuda")
    gq.bfs(qa, qb, d_off, d_cols, root, level, lanes, block, ctl)
    T.cuda.synchronize()
    assert qa.check_error() == gq.GQ_OK and qb.check_error() == gq.GQ_OK
    c = ctl.cpu().numpy()
    return level.cpu().numpy().view(np.uint32), int(c[160]), int(c[192])


def ymc_cells_for(nv, levels, lanes):
    return 4 * nv + (levels + 4) * lanes * 4 + (1 << 16)


def check(kind, off, cols, root, lanes, block=256):
    exp, nl, scanned = oracle.bfs(off, cols, root)
    print(f"[case] kind={kind} nv={len(off) - 1} m={len(cols)} root={root} lanes={lanes} "
          f"levels={nl}", flush=True)
    cells = ymc_cells_for(len(off) - 1, nl, lanes) if kind == "ymc" else 0
    got, levels, scanned_gpu = run_bfs(kind, off, cols, root, lanes, block, cells)
    assert np.array_equal(got, exp)
    assert levels == nl + 1 or levels == nl  # the last, empty level may be counted
    assert scanned_gpu == scanned  # every reached vertex's list is scanned once


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
@pytest.mark.parametrize("lanes", [256, 2048])
def test_bfs_small_graphs(kind, lanes):
    off, cols = workloads.grid_graph(64, 64)
    check(kind, off, cols, 0, lanes)
    check(kind, off, cols, 64 * 31 + 17, lanes)
    off, cols = workloads.rmat_graph(12, 16, seed=7)
    check(kind, off, cols, workloads.bfs_root(off, 7), lanes)
    # path plus isolated vertices, and a star with a hub of degree 1999
    off, cols = workloads._csr_from_pairs(300, np.arange(199), np.arange(1, 200))
    check(kind, off, cols, 5, lanes)
    off, cols = workloads._csr_from_pairs(2000, np.zeros(1999, dtype=np.int64), np.arange(1, 2000))
    check(kind, off, cols, 3, lanes)


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
def test_bfs_rmat22_full_size(kind):
    off, cols = workloads.rmat_graph(22, 16, seed=workloads.run_seed(4, 0))
    check(kind, off, cols, workloads.bfs_root(off, workloads.run_seed(4, 0)), 8192)


@pytest.mark.parametrize("kind", ["lfq"])
def test_bfs_grid4096_full_size(kind):
    off, cols = workloads.grid_graph(4096, 4096)
    rng = np.random.default_rng(workloads.run_seed(4, 1))
    check(kind, off, cols, int(rng.integers(0, 4096 * 4096)), 8192)
