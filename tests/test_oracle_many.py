"""The oracle's multi-threaded runner (orc_solve_many, used only to time the
oracle on the host cores) against its one-component search: every pass,
every thread count, every field.  A mistake in the runner's per-component
slicing of the concatenated inputs or outputs fails here."""
import os

import numpy as np
import pytest

import oracle
import workload
from algx_literal import random_graph
from oracle_cases import components
from workload.configs import CONFIGS


def check_many(sizes, edge_lists, k, budget):
    ref = [oracle.solve_component(n, e, k, budget) for n, e in zip(sizes, edge_lists)]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    per_pass = sum(r.nodes for r in ref)
    for threads in sorted({1, 2, os.cpu_count() or 1}):
        for passes in (1, 3):
            got = oracle.solve_many(sizes, edge_lists, k, budget, threads=threads, passes=passes)
            assert got["total_nodes"] == passes * per_pass, (threads, passes)
            for i, r in enumerate(ref):
                assert got["status"][i] == r.status, (threads, passes, i)
                assert got["nodes"][i] == r.nodes, (threads, passes, i)
                assert int(got["trace_hash"][i]) == r.trace_hash, (threads, passes, i)
                assert np.array_equal(got["colors"][offs[i]:offs[i + 1]], r.colors), (threads, i)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_solve_many_equals_solve_component_on_configs(cfg):
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    sizes, edge_lists, _ = components(g, w.k)
    assert len(sizes) > 0
    check_many(sizes, edge_lists, w.k, w.budget)


def test_solve_many_on_random_sets():
    rng = np.random.default_rng(5)
    for k in (2, 3, 4):
        sizes, edge_lists = [], []
        for _ in range(40):
            n = int(rng.integers(1, 30))
            e = random_graph(rng, n, float(rng.uniform(0.05, 0.5)))
            sizes.append(n)
            edge_lists.append(np.asarray(e, np.int32).reshape(-1, 2))
        check_many(sizes, edge_lists, k, 200)


def test_solve_many_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.solve_many([3], [np.array([[0, 1]], np.int32)], 3, 10, threads=0)
    with pytest.raises(ValueError):
        oracle.solve_many([3], [np.array([[0, 1]], np.int32)], 3, 10, threads=1, passes=0)
    r = oracle.solve_many([], [], 3, 10, threads=2)
    assert r["total_nodes"] == 0 and len(r["status"]) == 0
