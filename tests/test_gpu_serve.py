"""Serving: BFS jobs streamed through the persistent serving kernel
(include/gq_serve.h).  Every job's level hash must equal the hash of the CPU
BFS's levels (oracle O7), both when jobs overlap on the device and when each
runs alone; jobs are admitted by device-memory budget.

The level hash is the checksum defined in the header: the wrapping sum over
vertices v of splitmix64(seed, v) * (level[v] + 1)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import torch

pytestmark = pytest.mark.gpu


def level_hash(levels: np.ndarray) -> int:
    from paper_2606_01693_amd import SERVE_HASH_SEED
    v = np.arange(len(levels), dtype=np.uint64)
    with np.errstate(over="ignore"):
        w = workloads.splitmix64(SERVE_HASH_SEED, v)
        return int((w * (levels.astype(np.uint64) + np.uint64(1))).sum(dtype=np.uint64))


def path_graph(n):
    src = np.arange(n - 1, dtype=np.uint64)
    return workloads._csr_from_pairs(n, src, src + np.uint64(1))


def split_graph(n):
    """Two components: a star on the first half, a path on the second."""
    h = n // 2
    s1 = np.zeros(h - 1, dtype=np.uint64)
    d1 = np.arange(1, h, dtype=np.uint64)
    s2 = np.arange(h, n - 1, dtype=np.uint64)
    return workloads._csr_from_pairs(n, np.concatenate([s1, s2]),
                                     np.concatenate([d1, s2 + np.uint64(1)]))


def test_serve_levels_out_equal_cpu_bfs():
    """Each job alone, its levels written to a caller buffer: element-wise
    equal to the CPU BFS, and its hash equal to the hash of those levels."""
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(5, 100)
    pool = graph_pool(seed)
    outs = [T.full((p["nv"],), -7, dtype=T.int32, device="cuda") for p in pool]
    T.cuda.synchronize()
    reqs = [(p["off"], p["cols"], p["root"], o) for p, o in zip(pool, outs)]
    print(f"[case] serve levels_out jobs={len(reqs)}", flush=True)
    with gq.Server(teams=4, team_lanes=256, kind="lfq", budget_bytes=1 << 28, ring_slots=16,
                   idle_timeout_ms=20000) as srv:
        res = srv.run(reqs, np.zeros(len(reqs), dtype=np.int64), max_inflight=1)
    T.cuda.synchronize()
    for j, (p, o) in enumerate(zip(pool, outs)):
        got = o.cpu().numpy().view(np.uint32)
        exp, nl, _ = oracle.bfs(p["off"].cpu().numpy().view(np.uint32),
                                p["cols"].cpu().numpy().view(np.uint32), p["root"])
        diff = np.nonzero(got != exp)[0]
        assert len(diff) == 0, (f"job {j}: {len(diff)} levels differ, first {diff[:5]}: "
                                f"got {got[diff[:5]]} want {exp[diff[:5]]}")
        assert int(res["level_hash"][j]) == level_hash(got), (
            f"job {j}: device hash {int(res['level_hash'][j]):#x} != hash of its own levels "
            f"{level_hash(got):#x}")
        assert res["status"][j] == 0 and res["levels"][j] == nl


def graph_pool(seed):
    graphs = [path_graph(300), split_graph(512)]
    rng = np.random.default_rng(seed)
    for i, scale in enumerate(rng.integers(6, 13, size=6)):
        graphs.append(workloads.rmat_graph(int(scale), 16, seed=seed + i))
    pool = []
    T = torch()
    for j, (off, cols) in enumerate(graphs):
        root = workloads.bfs_root(off, seed + 17 * j)
        exp, nl, _ = oracle.bfs(off, cols, root)
        pool.append({"off": T.tensor(off.astype(np.int32), device="cuda"),
                     "cols": T.tensor(cols.astype(np.int32), device="cuda"),
                     "root": root, "hash": level_hash(exp), "levels": nl,
                     "nv": len(off) - 1, "nnz": len(cols)})
    T.cuda.synchronize()  # graphs resident before any server exists
    return pool


def jobs_from(pool, n, seed, mean_gap_ns):
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(pool), size=n)
    arrivals = np.cumsum(rng.exponential(mean_gap_ns, size=n)).astype(np.int64)
    reqs = [(pool[i]["off"], pool[i]["cols"], pool[i]["root"]) for i in pick]
    return pick, reqs, arrivals


def check(pool, pick, res):
    assert (res["status"] == 0).all(), res["status"]
    exp_hash = np.array([pool[i]["hash"] for i in pick], dtype=np.uint64)
    exp_lv = np.array([pool[i]["levels"] for i in pick])
    bad = np.nonzero(res["level_hash"] != exp_hash)[0]
    detail = [(int(b), int(pick[b]), hex(int(res["level_hash"][b])), hex(int(exp_hash[b])),
               int(res["levels"][b]), int(exp_lv[b])) for b in bad[:5]]
    assert len(bad) == 0, f"{len(bad)} jobs differ from the CPU BFS: {detail}"
    assert np.array_equal(res["levels"], exp_lv)
    assert (res["done_ns"] >= res["admit_ns"]).all()
    assert (res["admit_ns"] >= res["arrival_ns"]).all()


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
@pytest.mark.parametrize("team_lanes", [256, 1024])
def test_serve_mix_equals_alone_equals_oracle(kind, team_lanes):
    import paper_2606_01693_amd as gq
    seed = workloads.run_seed(5, 200)
    pool = graph_pool(seed)
    pick, reqs, arr = jobs_from(pool, 200, seed + 1, 20_000)
    print(f"[case] serve kind={kind} team_lanes={team_lanes} jobs={len(reqs)}", flush=True)
    with gq.Server(teams=32, team_lanes=team_lanes, kind=kind, budget_bytes=1 << 30,
                   ring_slots=256, idle_timeout_ms=20000) as srv:
        mix = srv.run(reqs, arr)
        check(pool, pick, mix)
        assert len(set(mix["team"].tolist())) > 1  # jobs really spread over teams
        # each distinct job alone
        alone_reqs = [(p["off"], p["cols"], p["root"]) for p in pool]
        alone = srv.run(alone_reqs, np.zeros(len(pool), dtype=np.int64), max_inflight=1)
        check(pool, np.arange(len(pool)), alone)


def test_serve_budget_admission():
    """A budget of 1.5x the second-largest job: jobs wait for memory, the
    largest job (larger than the whole budget) is refused, the rest stay
    exact, and the admitted bytes never exceed the budget."""
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(5, 300)
    pool = graph_pool(seed)
    off, cols = workloads.rmat_graph(14, 16, seed=seed + 99)
    root = workloads.bfs_root(off, seed)
    exp, nl, _ = oracle.bfs(off, cols, root)
    pool.append({"off": T.tensor(off.astype(np.int32), device="cuda"),
                 "cols": T.tensor(cols.astype(np.int32), device="cuda"), "root": root,
                 "hash": level_hash(exp), "levels": nl, "nv": len(off) - 1, "nnz": len(cols)})
    T.cuda.synchronize()
    with gq.Server(teams=8, team_lanes=256, kind="lfq", budget_bytes=1 << 26, ring_slots=16,
                   idle_timeout_ms=20000) as probe:
        jb = [probe.job_bytes(p["nv"], p["nnz"]) for p in pool]
    order = np.argsort(jb)
    budget = int(1.5 * jb[order[-2]])
    biggest = int(order[-1])
    assert jb[biggest] > budget
    with gq.Server(teams=16, team_lanes=256, kind="lfq", budget_bytes=budget, ring_slots=64,
                   idle_timeout_ms=20000) as srv:
        fits = [int(i) for i in order[:-1]]
        pick = np.array((fits * 8)[:48])
        reqs = [(pool[i]["off"], pool[i]["cols"], pool[i]["root"]) for i in pick]
        res = srv.run(reqs, np.zeros(len(reqs), dtype=np.int64))
        check(pool, pick, res)
        ev = sorted([(int(a), int(b)) for a, b in zip(res["admit_ns"], res["job_bytes"])] +
                    [(int(d), -int(b)) for d, b in zip(res["done_ns"], res["job_bytes"])],
                    key=lambda x: (x[0], x[1]))
        level = 0
        for _, b in ev:
            level += int(b)
            assert level <= budget
        r = srv.run([(pool[biggest]["off"], pool[biggest]["cols"], pool[biggest]["root"])],
                    np.zeros(1, dtype=np.int64))
        assert r["status"][0] == gq.GQ_ERR_NOMEM


def test_serve_start_stop_without_jobs():
    import paper_2606_01693_amd as gq
    with gq.Server(teams=8, team_lanes=64, kind="lfq", budget_bytes=1 << 24, ring_slots=16,
                   idle_timeout_ms=20000) as srv:
        r = srv.run([], np.zeros(0, dtype=np.int64))
        assert len(r["status"]) == 0


@pytest.mark.parametrize("kind", ["lfq", "wfq"])
def test_serve_mix_levels_elementwise_rmat12_20(kind):
    """The serving workload at its configured graph sizes: R-MAT scales 12..20
    (edge factor 16, one graph per scale), 120 jobs with Poisson arrivals
    overlapping on 64 teams of 1024 lanes, every job writing its levels to its
    own caller buffer.  Each job's levels equal the CPU BFS element by
    element, in the mix and with each graph's job alone."""
    import paper_2606_01693_amd as gq
    T = torch()
    seed = workloads.run_seed(5, 400)
    pool = []
    for i, scale in enumerate(range(12, 21)):
        off, cols = workloads.rmat_graph(scale, 16, seed=seed + i)
        root = workloads.bfs_root(off, seed + 31 * i)
        exp, nl, _ = oracle.bfs(off, cols, root)
        pool.append({"off": T.tensor(off.astype(np.int32), device="cuda"),
                     "cols": T.tensor(cols.astype(np.int32), device="cuda"), "root": root,
                     "exp": exp, "levels": nl, "nv": len(off) - 1})
    T.cuda.synchronize()
    rng = np.random.default_rng(seed + 1)
    pick = rng.integers(0, len(pool), size=120)
    arr = np.cumsum(rng.exponential(200_000, size=len(pick))).astype(np.int64)
    outs = [T.full((pool[i]["nv"],), -7, dtype=T.int32, device="cuda") for i in pick]
    reqs = [(pool[i]["off"], pool[i]["cols"], pool[i]["root"], o) for i, o in zip(pick, outs)]
    print(f"[case] serve element-wise kind={kind} jobs={len(reqs)} scales 12..20", flush=True)
    alone_outs = [T.full((p["nv"],), -7, dtype=T.int32, device="cuda") for p in pool]
    # both runs back to back: the server ends itself after its idle timeout
    with gq.Server(teams=64, team_lanes=1024, kind=kind, budget_bytes=8 << 30, ring_slots=256,
                   idle_timeout_ms=30000) as srv:
        mix = srv.run(reqs, arr)
        alone = srv.run([(p["off"], p["cols"], p["root"], o) for p, o in zip(pool, alone_outs)],
                        np.zeros(len(pool), dtype=np.int64), max_inflight=1)
    T.cuda.synchronize()
    assert (mix["status"] == 0).all(), mix["status"]
    assert len(set(mix["team"].tolist())) > 1
    for j, (i, o) in enumerate(zip(pick, outs)):
        got = o.cpu().numpy().view(np.uint32)
        diff = np.nonzero(got != pool[i]["exp"])[0]
        assert len(diff) == 0, f"mixed job {j} (scale {12 + i}): {len(diff)} levels differ"
        assert mix["levels"][j] == pool[i]["levels"]
    assert (alone["status"] == 0).all()
    for i, (p, o) in enumerate(zip(pool, alone_outs)):
        assert np.array_equal(o.cpu().numpy().view(np.uint32), p["exp"]), f"scale {12 + i}"
