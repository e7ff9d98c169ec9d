"""Pins of the oracle's exact-cover search (Sec. 2.3, Eq. 2, Algorithm 1).

* the exact-cover matrix against its closed-form shape and counts;
* feasibility against exhaustive k-coloring on tiny graphs;
* the exact-cover invariant on every solution;
* closed-form node counts (cliques, cycles) and hand-derived traces;
* status, node count, trace hash and colors against an independent
  set-based Algorithm X on random graphs, including every budget cut.
"""
import json
import os

import numpy as np
import pytest

import oracle
from algx_literal import (algx_sets, brute_force_colorable, complete, cycle,
                          trace_step, grotzsch, petersen, random_graph, wheel)

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def test_ec_matrix_shape_and_counts():
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = int(rng.integers(1, 9))
        k = int(rng.integers(2, 5))
        e = random_graph(rng, n, 0.5)
        M = oracle.ec_matrix(n, e, k).astype(np.int64)
        m = len(e)
        assert M.shape == (n * k, n + m * k)
        deg = np.zeros(n, int)
        for u, w in e:
            deg[u] += 1
            deg[w] += 1
        for v in range(n):
            for c in range(k):
                assert M[v * k + c].sum() == 1 + deg[v]
                assert M[v * k + c, v] == 1
        assert np.all(M[:, :n].sum(axis=0) == k)        # primary: k rows each
        assert np.all(M[:, n:].sum(axis=0) == 2)        # secondary: two ends
        assert M.sum() == n * k + 2 * m * k


def _check_exact_cover(n, e, k, colors):
    """Chosen rows (v, color[v]): every primary column once, every secondary
    column at most once."""
    M = oracle.ec_matrix(n, e, k).astype(np.int64)
    rows = [v * k + int(colors[v]) for v in range(n)]
    cover = M[rows].sum(axis=0)
    assert np.all(cover[:n] == 1)
    assert np.all(cover[n:] <= 1)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_feasibility_matches_brute_force(k):
    rng = np.random.default_rng(k)
    for trial in range(60):
        n = int(rng.integers(1, 9 if k < 4 else 8))
        e = random_graph(rng, n, float(rng.uniform(0.2, 0.9)))
        s = oracle.solve_component(n, e, k, 10**7)
        assert (s.status == oracle.FEASIBLE) == brute_force_colorable(n, e, k)
        if s.status == oracle.FEASIBLE:
            _check_exact_cover(n, e, k, s.colors)
            assert s.depth_at_stop == n
        else:
            assert np.all(s.colors == -1)


def test_closed_forms():
    cf = GOLDEN["closed_forms"]
    for k, nodes in cf["complete_infeasible"]:
        s = oracle.solve_component(k + 1, complete(k + 1), k, 10**7)
        assert (s.status, s.nodes) == (oracle.INFEASIBLE, nodes)
        # the count is the sum over levels of k!/(k-i)!
        import math
        assert nodes == sum(math.perm(k, i) for i in range(k + 1))
    for k in range(2, 7):
        s = oracle.solve_component(k, complete(k), k, 10**7)
        assert (s.status, s.nodes) == (oracle.FEASIBLE, k + 1)
        assert s.colors.tolist() == list(range(k))
    for n, nodes in cf["odd_cycle_k2"]:
        s = oracle.solve_component(n, cycle(n), 2, 10**7)
        assert (s.status, s.nodes) == (oracle.INFEASIBLE, nodes) == (1, 2 * n - 1)
    for n, nodes in cf["even_cycle_k2"]:
        s = oracle.solve_component(n, cycle(n), 2, 10**7)
        assert (s.status, s.nodes) == (oracle.FEASIBLE, nodes) == (0, n + 1)


def test_known_graphs():
    # Fig. 1b: a 4-clique is not 3-colorable
    assert oracle.solve_component(4, complete(4), 3, 10**6).status == oracle.INFEASIBLE
    assert oracle.solve_component(4, complete(4), 4, 10**6).status == oracle.FEASIBLE
    n, e = petersen()
    s = oracle.solve_component(n, e, 3, 10**6)
    assert s.status == oracle.FEASIBLE and brute_force_colorable(n, e, 3)
    _check_exact_cover(n, e, 3, s.colors)
    n, e = grotzsch()
    assert not brute_force_colorable(n, e, 3)
    assert oracle.solve_component(n, e, 3, 10**7).status == oracle.INFEASIBLE
    assert oracle.solve_component(n, e, 4, 10**7).status == oracle.FEASIBLE
    n, e = wheel(5)                      # odd wheel W5: chromatic number 4
    assert not brute_force_colorable(n, e, 3)
    assert oracle.solve_component(n, e, 3, 10**7).status == oracle.INFEASIBLE
    n, e = wheel(6)                      # even wheel: 3-colorable
    assert oracle.solve_component(n, e, 3, 10**7).status == oracle.FEASIBLE


@pytest.mark.parametrize("case", GOLDEN["traces"], ids=lambda c: c["name"])
def test_hand_traces(case):
    s = oracle.solve_component(case["n"], case["edges"], case["k"], 10**6)
    h = 0
    for rec in case["trace"]:
        h = trace_step(h, rec)
    assert s.status == case["status"]
    assert s.nodes == len(case["trace"])
    assert s.trace_hash == h, case["why"]
    if "colors" in case:
        assert s.colors.tolist() == case["colors"]


def test_budget_boundary_k4():
    for b in range(1, 25):
        s = oracle.solve_component(4, complete(4), 3, b)
        if b >= 16:
            assert (s.status, s.nodes) == (oracle.INFEASIBLE, 16)
        else:
            assert (s.status, s.nodes) == (oracle.BUDGET, b)
            assert np.all(s.colors == -1)


def _same(a, b):
    status, nodes, h, depth, colors = b
    assert a.status == status
    assert a.nodes == nodes
    assert a.trace_hash == h
    assert a.depth_at_stop == depth
    assert a.colors.tolist() == colors.tolist()


@pytest.mark.parametrize("k", [2, 3, 4])
def test_matches_set_based_algorithm_x(k):
    rng = np.random.default_rng(100 + k)
    for trial in range(80):
        n = int(rng.integers(1, 16))
        # around the k-colorability threshold, where the search backtracks
        p = float(rng.uniform(0.15, 0.6)) * (k / 3.0)
        e = random_graph(rng, n, min(p, 0.95))
        ref = algx_sets(n, e, k, 10**6)
        _same(oracle.solve_component(n, e, k, 10**6), ref)


def test_matches_set_based_algorithm_x_every_budget():
    rng = np.random.default_rng(7)
    for trial in range(12):
        n = int(rng.integers(6, 13))
        e = random_graph(rng, n, 0.45)
        full = algx_sets(n, e, 3, 10**6)
        for b in range(1, full[1] + 2):
            _same(oracle.solve_component(n, e, 3, b), algx_sets(n, e, 3, b))


def test_relabelling_changes_trace_not_feasibility():
    """The search is deterministic in the local numbering: the same graph
    under another numbering keeps feasibility but may take another path."""
    n, e = petersen()
    base = oracle.solve_component(n, e, 3, 10**6)
    perm = np.random.default_rng(1).permutation(n)
    e2 = [(int(perm[u]), int(perm[w])) for u, w in e]
    other = oracle.solve_component(n, e2, 3, 10**6)
    assert other.status == base.status == oracle.FEASIBLE
    _check_exact_cover(n, e2, 3, other.colors)
