"""Pins of the oracle's stitch-aware row order (Eq. 1 counts a stitch for
each pair of split halves colored differently; reading: a column whose
node's stitch partner is already colored on the path tries that color's
row first, the other rows ascending).

* status, node count, trace hash, depth and colors equal an independent
  set-based Algorithm X with the same order, on random graphs with random
  partner pairs and at budget cuts;
* without partners it is the plain search; every solution is a proper
  coloring (the exact-cover invariant);
* a hand case where the order keeps two halves alike that the plain order
  splits; in the whole flow on the stitch workload it never changes
  feasibility and lowers the stitch count.
"""
import numpy as np
import pytest

import oracle
from algx_literal import algx_sets, random_graph


def random_partners(rng, n, edges, pairs):
    adj = set(map(tuple, edges)) | {(b, a) for a, b in edges}
    part = [-1] * n
    for _ in range(pairs * 4):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b and part[a] < 0 and part[b] < 0 and (a, b) not in adj:
            part[a], part[b] = b, a
    return part


def same(got, ref):
    st, nodes, h, depth, colors = ref
    assert (got.status, got.nodes, got.trace_hash, got.depth_at_stop) == (st, nodes, h, depth)
    assert np.array_equal(got.colors, colors)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_matches_set_based_order(k):
    rng = np.random.default_rng(900 + k)
    for _ in range(80):
        n = int(rng.integers(2, 16))
        e = random_graph(rng, n, min(0.9, float(rng.uniform(0.15, 0.6)) * k / 3.0))
        part = random_partners(rng, n, e, n // 3)
        same(oracle.solve_component(n, e, k, 10**6, part), algx_sets(n, e, k, 10**6, part))


def test_every_budget_cut():
    rng = np.random.default_rng(17)
    for _ in range(10):
        n = int(rng.integers(6, 13))
        e = random_graph(rng, n, 0.45)
        part = random_partners(rng, n, e, 4)
        full = algx_sets(n, e, 3, 10**6, part)
        for b in range(1, full[1] + 2):
            same(oracle.solve_component(n, e, 3, b, part), algx_sets(n, e, 3, b, part))


def test_no_partner_is_the_plain_search_and_solutions_are_proper():
    rng = np.random.default_rng(23)
    for _ in range(60):
        n = int(rng.integers(2, 20))
        e = random_graph(rng, n, 0.3)
        plain = oracle.solve_component(n, e, 3, 10**6)
        none = oracle.solve_component(n, e, 3, 10**6, [-1] * n)
        assert (plain.status, plain.nodes, plain.trace_hash) == (none.status, none.nodes, none.trace_hash)
        part = random_partners(rng, n, e, n // 3)
        s = oracle.solve_component(n, e, 3, 10**6, part)
        if s.status == oracle.FEASIBLE:
            assert (s.colors >= 0).all()
            assert all(s.colors[a] != s.colors[b] for a, b in e)


def test_hand_case_keeps_halves_alike():
    # triangle 0-1-2 with pendant 3 on 1 and pendant 4 on 0, k = 3, halves
    # 2 and 3 (not adjacent): the plain order gives 0, 1, 2 to the triangle
    # and node 3 takes its lowest open color 0; with the order node 3 takes
    # its partner's color 2, which is still open at 3
    n, e = 5, [(0, 1), (0, 2), (1, 2), (1, 3), (0, 4)]
    part = [-1, -1, 3, 2, -1]
    plain = oracle.solve_component(n, e, 3, 10**6)
    st = oracle.solve_component(n, e, 3, 10**6, part)
    assert plain.status == st.status == oracle.FEASIBLE
    assert plain.colors[2] != plain.colors[3]
    assert st.colors[2] == st.colors[3]


def test_whole_flow_fewer_stitches():
    import workload
    from workload.configs import CONFIGS
    w = CONFIGS[2]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    plain = oracle.decompose(g, w.k, w.budget)
    st = oracle.decompose(g, w.k, w.budget, stitch=True)
    assert np.array_equal(plain.comps["status"], st.comps["status"])
    inside = lambda d: int(d.comps["stitches"][d.comps["stitches"] > 0].sum())
    assert inside(st) < inside(plain) // 4     # stitches inside solved components
    assert st.stitches < plain.stitches and st.conflicts == 0
