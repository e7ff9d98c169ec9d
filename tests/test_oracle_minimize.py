"""Pins of the oracle's Eq. 1 minimisation (orc_minimize_component and the
ORC_MINIMIZE flow): exact least cost against exhaustive search on tiny
graphs, closed forms, an independent restatement of the branch and bound
(node counts, stop flag, colors), budget behaviour and the flow's
bookkeeping.  Cost = 10 conflicts + stitches (Eq. 1, alpha = 0.1)."""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import bb_sets, complete, cycle, eq1_cost, min_eq1_cost, random_graph
from oracle_cases import components
from workload.configs import CONFIGS


def random_partner(rng, n, frac, edges):
    """Disjoint stitch pairs that are not conflict pairs."""
    es = {(min(u, w), max(u, w)) for u, w in edges}
    part = [-1] * n
    perm = rng.permutation(n)
    for i in range(0, n - 1, 2):
        a, b = int(perm[i]), int(perm[i + 1])
        if rng.random() < frac and (min(a, b), max(a, b)) not in es:
            part[a], part[b] = b, a
    return part


def incumbent(n, edges, k):
    s = oracle.solve_component(n, edges, k, 10**6)
    return s.colors if s.status == oracle.FEASIBLE else oracle.mark_conflicts(n, edges, k)


def test_closed_forms():
    # K_{k+1}: one conflict is unavoidable
    for k in (2, 3, 4):
        n = k + 1
        r = oracle.minimize_component(n, complete(n), k, incumbent(n, complete(n), k), 10**6)
        assert r.cost == 10 and not r.stopped and eq1_cost(n, complete(n), r.colors) == 10
    # K5, k = 3: classes 2, 2, 1 -> two conflicts (Turan)
    r = oracle.minimize_component(5, complete(5), 3, incumbent(5, complete(5), 3), 10**6)
    assert r.cost == 20
    # K7, k = 3: classes 3, 2, 2 -> 3 + 1 + 1 = 5 conflicts
    r = oracle.minimize_component(7, complete(7), 3, incumbent(7, complete(7), 3), 10**6)
    assert r.cost == 50
    # odd cycle with two colors: one conflict
    r = oracle.minimize_component(7, cycle(7), 2, incumbent(7, cycle(7), 2), 10**6)
    assert r.cost == 10
    # a forced stitch: k = 2, 2-3 adjacent, 0-2 and 1-3 adjacent, 0 and 1
    # stitch partners -> 0 and 1 must differ: least cost 1 (one stitch)
    e = [(0, 2), (1, 3), (2, 3)]
    part = [1, 0, -1, -1]
    r = oracle.minimize_component(4, e, 2, [0, 0, 1, 0], 10**6, part)   # incumbent: 1 conflict
    assert r.cost == 1 and eq1_cost(4, e, r.colors, part) == 1
    # a cost-0 incumbent is left alone
    r = oracle.minimize_component(3, complete(3), 3, [0, 1, 2], 10**6)
    assert (r.nodes, r.cost, list(r.colors)) == (0, 0, [0, 1, 2])


@pytest.mark.parametrize("k", [2, 3, 4])
def test_least_cost_equals_exhaustive_search(k):
    rng = np.random.default_rng(40 + k)
    checked = 0
    for _ in range(60):
        n = int(rng.integers(2, 10 if k < 4 else 8))
        e = random_graph(rng, n, float(rng.uniform(0.3, 0.9)))
        part = random_partner(rng, n, 0.6, e)
        inc = incumbent(n, e, k)
        r = oracle.minimize_component(n, e, k, inc, 10**7, part)
        assert not r.stopped
        assert r.cost == eq1_cost(n, e, r.colors, part)
        assert r.cost <= eq1_cost(n, e, inc, part)
        assert r.cost == min_eq1_cost(n, e, k, part), (n, e, k, part)
        checked += r.nodes > 0
    assert checked > 10


@pytest.mark.parametrize("k", [2, 3, 4])
def test_branch_and_bound_equals_restatement(k):
    """Node counts, stop flag, colors and cost equal the set-based
    restatement at full budget and at budget cuts."""
    rng = np.random.default_rng(70 + k)
    for _ in range(40):
        n = int(rng.integers(2, 22))
        e = random_graph(rng, n, float(rng.uniform(1.2, 2.2)) * k / n)
        part = random_partner(rng, n, 0.5, e)
        inc = incumbent(n, e, k)
        for budget in (1, 2, 5, 17, 100, 10**5):
            r = oracle.minimize_component(n, e, k, inc, budget, part)
            c, nodes, stopped, cost = bb_sets(n, e, k, inc, budget, part)
            assert (r.nodes, r.stopped, r.cost) == (nodes, stopped, cost), (n, e, k, budget)
            assert np.array_equal(r.colors, c)
            if r.stopped:
                assert r.nodes == budget


def test_budget_is_monotone_and_exact():
    rng = np.random.default_rng(3)
    n = 18
    e = random_graph(rng, n, 0.35)
    inc = incumbent(n, e, 3)
    full = oracle.minimize_component(n, e, 3, inc, 10**7)
    assert not full.stopped
    last = eq1_cost(n, e, inc)
    for b in range(1, full.nodes + 2):
        r = oracle.minimize_component(n, e, 3, inc, b)
        assert r.cost <= last            # more budget never costs more
        last = r.cost
        if b < full.nodes:
            assert r.stopped and r.nodes == b
        else:
            assert not r.stopped and r.nodes == full.nodes and r.cost == full.cost
    assert last == full.cost


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.minimize_component(3, [(0, 1)], 3, [0, -1, 0], 10)       # incomplete incumbent
    with pytest.raises(ValueError):
        oracle.minimize_component(3, [(0, 1)], 3, [0, 1, 0], 10, [1, -1, -1])   # asymmetric
    with pytest.raises(ValueError):
        oracle.minimize_component(3, [(0, 1)], 3, [0, 1, 0], 0)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_flow_minimizes_every_small_component(cfg):
    """ORC_MINIMIZE in the whole flow: search status and node counts stay
    the search's, every component of at most 64 nodes with a positive cost
    is minimised (its record carries the branch-and-bound node count, its
    colors equal orc_minimize_component's from the same incumbent), larger
    ones keep the marking; no cost rises."""
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    mb = 2000
    base = oracle.decompose(g, w.k, w.budget, mark=True)
    got = oracle.decompose(g, w.k, w.budget, minimize=True, min_budget=mb)
    for f in ("status", "nodes", "size"):
        assert np.array_equal(got.comps[f], base.comps[f])
    assert got.conflicts <= base.conflicts
    _, comp_of, comps = oracle.simplify(g, w.k)
    partner = np.full(g.num_nodes, -1, np.int64)
    for a, b in g.se.tolist():
        partner[a], partner[b] = b, a
    sizes, edge_lists, members = components(g, w.k)
    ran = 0
    for i, (n, e, mem) in enumerate(zip(sizes, edge_lists, members)):
        loc = {int(v): j for j, v in enumerate(mem.tolist())}
        lp = [loc.get(int(partner[v]), -1) if partner[v] >= 0 else -1 for v in mem.tolist()]
        inc = base.colors[mem]
        rec = got.comps[i]
        before = eq1_cost(n, e.tolist(), inc, lp)
        after = eq1_cost(n, e.tolist(), got.colors[mem], lp)
        assert after <= before
        if n <= oracle.MINIMIZE_MAX_N and before > 0:
            r = oracle.minimize_component(n, e, w.k, inc, mb, lp)
            assert np.array_equal(got.colors[mem], r.colors)
            assert rec["min_nodes"] == (-r.nodes if r.stopped else r.nodes)
            ran += 1
        else:
            assert rec["min_nodes"] == 0
            assert np.array_equal(got.colors[mem], inc)
    assert ran > 0
