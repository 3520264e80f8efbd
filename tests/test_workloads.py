"""The fast C graph builders produce exactly the graphs the numpy definitions
in workloads/ produce (CPU only)."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("scale,seed", [(8, 1), (11, 5), (12, 9)])
def test_rmat_fast_equals_definition(scale, seed):
    a = workloads.rmat_graph(scale, 16, seed=seed, fast=True)
    b = workloads.rmat_graph(scale, 16, seed=seed, fast=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("rows,cols", [(1, 9), (7, 3), (50, 70), (129, 64)])
def test_grid_fast_equals_definition(rows, cols):
    a = workloads.grid_graph(rows, cols, fast=True)
    b = workloads.grid_graph(rows, cols, fast=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_grid_edge_count_closed_form():
    off, cols = workloads.grid_graph(33, 47)
    # undirected edges 33*46 + 32*47, each stored twice
    assert len(cols) == 2 * (33 * 46 + 32 * 47)
    assert off[-1] == len(cols)


def test_mix_roles_are_fair_coin():
    r = workloads.mix_roles(123, 1024, 256)
    assert abs(r.mean() - 0.5) < 0.01
