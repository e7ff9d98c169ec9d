"""Pins of the oracle's layout graph, simplification, sub-graphs, recovery.

The layout graph (Sec. 2.1) is checked against an exhaustive O(N^2) pair
test and against hand-computed rectangle pairs; simplification and
components against networkx and a hand-derived FIFO example; recovery
against its invariants and the closed form on K_k.
"""
import json
import os

import networkx as nx
import numpy as np
import pytest

import oracle
import workload

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def brute_edges(nodes, dmin, partner):
    """All pairs, gap of closed boxes, strict < dmin; stitch pairs excluded."""
    n = len(nodes)
    out = []
    x0, y0, x1, y1 = (nodes[:, i].astype(np.int64) for i in range(4))
    for i in range(n):
        gx = np.maximum(0, np.maximum(x0[i + 1:] - x1[i], x0[i] - x1[i + 1:]))
        gy = np.maximum(0, np.maximum(y0[i + 1:] - y1[i], y0[i] - y1[i + 1:]))
        hit = np.nonzero(gx * gx + gy * gy < dmin * dmin)[0] + i + 1
        for j in hit:
            if partner.get(i) != j:
                out.append((i, int(j)))
    return sorted(out)


def split_nodes(rects, split_len):
    nodes, partner = [], {}
    for x0, y0, x1, y1 in rects.tolist():
        w, h = x1 - x0, y1 - y0
        L = max(w, h)
        if split_len and L > split_len:
            m = L // 2
            if w >= h:
                a, b = [x0, y0, x0 + m, y1], [x0 + m, y0, x1, y1]
            else:
                a, b = [x0, y0, x1, y0 + m], [x0, y0 + m, x1, y1]
            partner[len(nodes)] = len(nodes) + 1
            partner[len(nodes) + 1] = len(nodes)
            nodes += [a, b]
        else:
            nodes.append([x0, y0, x1, y1])
    return np.asarray(nodes, dtype=np.int64).reshape(-1, 4), partner


@pytest.mark.parametrize("case", GOLDEN["rect_pairs"])
def test_hand_rect_pairs(case):
    g = oracle.build_graph(np.array([case["a"], case["b"]]), case["dmin"])
    assert (len(g.ce) == 1) == case["edge"], case["why"]


@pytest.mark.parametrize("case", GOLDEN["split_cases"])
def test_hand_split(case):
    # a lone rectangle: its halves are nodes 0 and 1 joined by one stitch edge
    g = oracle.build_graph(np.array([case["rect"]]), 80, case["split_len"])
    assert g.num_nodes == len(case["halves"])
    assert len(g.ce) == 0
    assert len(g.se) == (1 if len(case["halves"]) == 2 else 0)
    nodes, _ = split_nodes(np.array([case["rect"]]), case["split_len"])
    assert nodes.tolist() == case["halves"], case["why"]


@pytest.mark.parametrize("n,side,dmin,split", [(1500, 3000, 80, 0), (2500, 6000, 120, 120),
                                               (800, 1500, 100, 0), (3000, 9000, 80, 0)])
def test_conflict_graph_matches_all_pairs(n, side, dmin, split):
    rects, _ = workload.generate(n, side, seed=n)
    g = oracle.build_graph(rects, dmin, split)
    nodes, partner = split_nodes(rects, split)
    assert g.num_nodes == len(nodes)
    assert [tuple(e) for e in g.ce.tolist()] == brute_edges(nodes, dmin, partner)
    assert sorted(tuple(p) for p in g.se.tolist()) == sorted(
        (a, b) for a, b in partner.items() if a < b)


def test_fifo_example():
    ex = GOLDEN["fifo_example"]
    g = oracle.Graph(ex["num_nodes"], np.array(sorted(tuple(sorted(e)) for e in ex["edges"])),
                     np.zeros((0, 2), np.int32))
    rem, comp_of, comps = oracle.simplify(g, ex["k"])
    assert rem.tolist() == ex["removal_order"], ex["why"]
    assert [c.tolist() for c in comps] == ex["components_local_order"]
    d = oracle.decompose(g, ex["k"], 10**6)
    assert d.comps["status"].tolist() == [ex["search"]["status"]]
    assert d.comps["nodes"].tolist() == [ex["search"]["nodes"]]
    assert d.colors.tolist() == ex["colors_after_recovery"]


def test_bfs_example():
    ex = GOLDEN["bfs_example"]
    g = oracle.Graph(ex["num_nodes"], np.array(sorted(tuple(sorted(e)) for e in ex["edges"])),
                     np.zeros((0, 2), np.int32))
    rem, _, comps = oracle.simplify(g, ex["k"])
    assert len(rem) == 0
    assert [c.tolist() for c in comps] == [ex["local_order"]], ex["why"]


def _nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.num_nodes))
    G.add_edges_from(map(tuple, g.ce.tolist()))
    return G


@pytest.mark.parametrize("k,dmin,side,split", [(3, 80, 3000, 0), (3, 100, 3000, 0),
                                               (4, 120, 4000, 120)])
def test_kcore_and_components_match_networkx(k, dmin, side, split):
    rects, _ = workload.generate(1500, side, seed=k * 1000 + dmin)
    g = oracle.build_graph(rects, dmin, split)
    rem, comp_of, comps = oracle.simplify(g, k)
    G = _nx_graph(g)
    core = set(nx.k_core(G, k).nodes())
    assert core == set(np.nonzero(comp_of >= 0)[0].tolist())
    assert set(rem.tolist()) == set(range(g.num_nodes)) - core
    assert len(rem) == len(set(rem.tolist()))
    ref = sorted(sorted(c) for c in nx.connected_components(G.subgraph(core)))
    ours = sorted(sorted(c.tolist()) for c in comps)
    assert ours == ref
    # ordered by smallest id; each starts at its smallest id; min degree >= k
    firsts = [int(c[0]) for c in comps]
    assert firsts == sorted(firsts)
    for c in comps:
        assert int(c[0]) == int(c.min())
        assert len(c) >= k + 1
        H = G.subgraph(c.tolist())
        assert min(dict(H.degree()).values()) >= k


def test_fifo_order_is_a_valid_peeling():
    """Every removed node has < k neighbours among the nodes removed after it
    plus the core (the property recovery relies on)."""
    rects, _ = workload.generate(2000, 3500, seed=11)
    g = oracle.build_graph(rects, 80)
    k = 3
    rem, comp_of, _ = oracle.simplify(g, k)
    G = _nx_graph(g)
    pos = {v: i for i, v in enumerate(rem.tolist())}
    for v in rem.tolist():
        later = [w for w in G[v] if pos.get(w, 1 << 30) > pos[v]]
        assert len(later) < k


def test_recovery_invariants_and_closed_form():
    # K_k with k colors: removed whole; reverse FIFO gives color k-1-i
    for k in (2, 3, 4, 5):
        e = np.array([(i, j) for i in range(k) for j in range(i + 1, k)], np.int32)
        d = oracle.decompose(oracle.Graph(k, e, np.zeros((0, 2), np.int32)), k, 100)
        assert d.colors.tolist() == [k - 1 - i for i in range(k)]
        assert len(d.comps) == 0
    # random layouts: recovered nodes never conflict with colored neighbours
    for seed in range(4):
        rects, _ = workload.generate(1200, 2600, seed=seed)
        g = oracle.build_graph(rects, 90)
        d = oracle.decompose(g, 3, 10**5)
        c = d.colors
        assert d.conflicts == 0
        a, b = g.ce[:, 0], g.ce[:, 1]
        both = (c[a] >= 0) & (c[b] >= 0)
        assert not np.any(c[a][both] == c[b][both])
        removed = d.comp_of < 0
        assert np.all(c[removed] >= 0)
        assert d.uncolored == int(np.sum(c < 0))


def test_stitch_partner_preference_and_counts():
    # Halves 0 = [0,100]x[0,20], 1 = [100,200]x[0,20] of one rectangle and a
    # neighbour 2; all three have degree < 3, FIFO removal order 0, 1, 2,
    # recovery runs 2, 1, 0.
    # (a) neighbour next to the right half: 2 -> 0; 1 sees 2 -> 1; 0 takes
    #     its partner's color 1 (no neighbour uses it): no stitch.
    g = oracle.build_graph(np.array([[0, 0, 200, 20], [180, 60, 200, 100]]), 80, 120)
    assert g.num_nodes == 3 and g.se.tolist() == [[0, 1]] and g.ce.tolist() == [[1, 2]]
    d = oracle.decompose(g, 3, 100)
    assert d.colors.tolist() == [1, 1, 0] and d.stitches == 0
    # (b) neighbour next to the left half: 2 -> 0; 1 has no colored neighbour
    #     -> 0; 0 may not take 0 (used by 2) -> 1: one stitch.
    g = oracle.build_graph(np.array([[0, 0, 200, 20], [0, 60, 20, 100]]), 80, 120)
    assert g.ce.tolist() == [[0, 2]]
    d = oracle.decompose(g, 3, 100)
    assert d.colors.tolist() == [1, 0, 0] and d.stitches == 1
    # recount stitches from colors on a stitched random layout
    rects, _ = workload.generate(3000, 5000, seed=5)
    g = oracle.build_graph(rects, 120, 120)
    d = oracle.decompose(g, 4, 10**4)
    c = d.colors
    s = g.se
    ok = (c[s[:, 0]] >= 0) & (c[s[:, 1]] >= 0)
    assert d.stitches == int(np.sum(ok & (c[s[:, 0]] != c[s[:, 1]])))
    for ci, rec in enumerate(d.comps):
        inside = (d.comp_of[s[:, 0]] == ci) & (d.comp_of[s[:, 1]] == ci)
        if rec["status"] == oracle.FEASIBLE:
            assert rec["stitches"] == int(np.sum(inside & (c[s[:, 0]] != c[s[:, 1]])))
        else:
            assert rec["stitches"] == -1


def test_invalid_inputs_rejected():
    bad = [np.array([[0, 0]]), np.array([[0, 5]]), np.array([[0, 1], [0, 1]])]
    for e in bad:
        with pytest.raises(ValueError):
            oracle.decompose(oracle.Graph(3, e, np.zeros((0, 2), np.int32)), 3, 10)
    with pytest.raises(ValueError):   # a pair both stitch and conflict
        oracle.decompose(oracle.Graph(2, np.array([[0, 1]]), np.array([[0, 1]])), 3, 10)
