"""Pins of the oracle's conflict marking (Algorithm 1: a column left with
no related row is a conflict candidate (cl, cl'), cl' the column whose
cover removed cl's final row).  Reading: one descent of the search without
backtracking, in which such a column takes the row it lost last.

* closed forms: K_{k+1} with k colors keeps exactly one conflict, between
  its last two nodes; an odd cycle with 2 colors keeps one, an even cycle
  and K_k none;
* every node is colored, every conflict touches a marked node, and the
  count is never below the exhaustive minimum over all k-colorings;
* the colors equal those of an independent set-based descent;
* in the whole flow: feasible components are untouched, the others are
  fully colored, and the per-component and total conflicts are the
  monochromatic conflict edges (recovery adds none).
"""
import numpy as np
import pytest

import oracle
from algx_literal import (complete, cycle, grotzsch, mark_sets, min_conflicts, petersen,
                          random_graph, wheel)


def conflicts(colors, edges):
    return sum(1 for u, w in edges if colors[u] == colors[w])


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_clique_one_more_than_k(k):
    n = k + 1
    e = complete(n)
    c = oracle.mark_conflicts(n, e, k)
    assert (c >= 0).all() and (c < k).all()
    assert conflicts(c, e) == 1
    # nodes 0 .. k-1 take colors 0 .. k-1; node k lost color k-1 last
    assert list(c) == list(range(k)) + [k - 1]


@pytest.mark.parametrize("n", [3, 5, 7, 9, 11])
def test_odd_cycle_two_colors(n):
    e = cycle(n)
    c = oracle.mark_conflicts(n, e, 2)
    assert conflicts(c, e) == 1
    assert min_conflicts(n, e, 2) == 1


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_even_cycle_and_small_clique_no_conflict(n):
    assert conflicts(oracle.mark_conflicts(n, cycle(n), 2), cycle(n)) == 0
    k = n // 2
    assert conflicts(oracle.mark_conflicts(k, complete(k), k), complete(k)) == 0


def test_known_graphs_at_least_the_minimum():
    for (n, e), k in ((petersen(), 3), (grotzsch(), 3), (wheel(5), 3), (wheel(6), 3)):
        c = oracle.mark_conflicts(n, e, k)
        assert (c >= 0).all()
        assert conflicts(c, e) >= min_conflicts(n, e, k)


@pytest.mark.parametrize("k", [2, 3])
def test_never_below_exhaustive_minimum(k):
    rng = np.random.default_rng(40 + k)
    for _ in range(60):
        n = int(rng.integers(2, 9))
        e = random_graph(rng, n, float(rng.uniform(0.3, 0.9)))
        c = oracle.mark_conflicts(n, e, k)
        assert (c >= 0).all() and (c < k).all()
        assert conflicts(c, e) >= min_conflicts(n, e, k)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
def test_matches_set_based_descent(k):
    rng = np.random.default_rng(500 + k)
    for _ in range(60):
        n = int(rng.integers(1, 40))
        p = min(0.95, float(rng.uniform(0.3, 2.0)) * 2.0 * k / max(n, 1))
        e = random_graph(rng, n, p)
        assert np.array_equal(oracle.mark_conflicts(n, e, k), mark_sets(n, e, k)), (n, k, e)


def test_whole_flow_marks_only_failed_components():
    import workload
    from workload.configs import CONFIGS
    w = CONFIGS[0]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    plain = oracle.decompose(g, w.k, w.budget)
    marked = oracle.decompose(g, w.k, w.budget, mark=True)
    assert (plain.comps["status"] != oracle.FEASIBLE).any()
    assert marked.uncolored == 0
    for f in ("size", "status", "nodes", "trace_hash", "depth_at_stop", "first_node", "num_edges"):
        assert np.array_equal(plain.comps[f], marked.comps[f])
    feas = plain.comp_of >= 0
    feas &= plain.comps["status"][np.maximum(plain.comp_of, 0)] == oracle.FEASIBLE
    assert np.array_equal(plain.colors[feas], marked.colors[feas])
    ce = g.ce
    same = marked.colors[ce[:, 0]] == marked.colors[ce[:, 1]]
    assert marked.conflicts == int(same.sum()) == int(marked.comps["conflicts"].sum()) > 0
    assert plain.conflicts == 0 and (plain.comps["conflicts"] == 0).all()
    # each component's conflicts are the monochromatic edges inside it
    for ci, rec in enumerate(marked.comps):
        inside = (marked.comp_of[ce[:, 0]] == ci) & (marked.comp_of[ce[:, 1]] == ci)
        assert rec["conflicts"] == int((same & inside).sum())
        assert rec["stitches"] >= 0
