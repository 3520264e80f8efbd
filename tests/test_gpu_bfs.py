"""Queue-driven BFS on the GPU: levels must equal the CPU BFS (oracle O7)
bit-exactly, on small graphs and on the full-size R-MAT (scale 22) and
4096 x 4096 grid inputs."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import torch

pytestmark = pytest.mark.gpu


def run_bfs(kind, off, cols, root, lanes, block=256, ymc_cells=0, ctl_bytes=None):
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
    if ctl_bytes is None:
        ctl_bytes = gq.bfs_ctl_bytes(len(cols))
    ctl = T.zeros(ctl_bytes // 8, dtype=T.int64, device="cuda")
    gq.bfs(qa, qb, d_off, d_cols, root, level, lanes, block, ctl)
    T.cuda.synchronize()
    assert qa.check_error() == gq.GQ_OK and qb.check_error() == gq.GQ_OK
    c = ctl.cpu().numpy()
    return level.cpu().numpy().view(np.uint32), int(c[160]), int(c[192])


def ymc_cells_for(nv, levels, lanes):
    return 4 * nv + (levels + 4) * lanes * 4 + (1 << 16)


def check(kind, off, cols, root, lanes, block=256, ctl_bytes=None):
    exp, nl, scanned = oracle.bfs(off, cols, root)
    print(f"[case] kind={kind} nv={len(off) - 1} m={len(cols)} root={root} lanes={lanes} "
          f"levels={nl} ctl_bytes={ctl_bytes}", flush=True)
    cells = ymc_cells_for(len(off) - 1, nl, lanes) if kind == "ymc" else 0
    got, levels, scanned_gpu = run_bfs(kind, off, cols, root, lanes, block, cells, ctl_bytes)
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


def stars(nv, centres, degree, seed):
    """Star hubs of the given degree around `centres`, chained together, plus
    a sparse random graph on the rest: many vertices of degree >= 1024 in one
    level."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for i, c in enumerate(centres):
        leaves = rng.choice(nv, size=degree, replace=False)
        src.append(np.full(degree, c))
        dst.append(leaves)
        if i:
            src.append(np.array([centres[i - 1]]))
            dst.append(np.array([c]))
    src.append(rng.integers(0, nv, size=4 * nv))
    dst.append(rng.integers(0, nv, size=4 * nv))
    return workloads._csr_from_pairs(nv, np.concatenate(src), np.concatenate(dst))


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
@pytest.mark.parametrize("ctl_kib", [4, 5, None])
def test_bfs_hub_lists(kind, ctl_kib):
    """Vertices of degree >= 1024 split over all wavefronts: with the full hub
    list (None), with room for 128 hubs (5 KiB: the rest scanned by their own
    wavefront) and with none (4 KiB)."""
    off, cols = stars(1 << 15, list(range(0, 4000, 13)), 1500, 11)
    check(kind, off, cols, 0, 4096, ctl_bytes=None if ctl_kib is None else ctl_kib * 1024)


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_bfs_rmat22_full_size(kind):
    off, cols = workloads.rmat_graph(22, 16, seed=workloads.run_seed(4, 0))
    check(kind, off, cols, workloads.bfs_root(off, workloads.run_seed(4, 0)), 8192)


@pytest.mark.parametrize("kind", ["lfq", "wfq", "ymc"])
def test_bfs_grid4096_full_size(kind):
    off, cols = workloads.grid_graph(4096, 4096)
    rng = np.random.default_rng(workloads.run_seed(4, 1))
    check(kind, off, cols, int(rng.integers(0, 4096 * 4096)), 8192)
