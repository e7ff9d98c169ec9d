"""Device simplification and sub-graph split (mpld_split_graph_device;
Sec. 2.2 simplification, Algorithm 1's sub-graphs) against the oracle's
sequential definitions: FIFO removal order, components ordered by smallest
id and BFS local numbering must be identical, element by element.
"""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import random_graph
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def check(ctx, n, ce, k, simplify=True):
    import paper_2303_14335_amd as mp
    ce = np.ascontiguousarray(np.asarray(ce, dtype=np.int32).reshape(-1, 2))
    se = np.zeros((0, 2), np.int32)
    rem, comp_of, comps = oracle.simplify(oracle.Graph(n, ce, se), k, simplify)
    grem, gcomp_of, gcomps = mp.mpld_split_graph_device(ctx, mp.Graph(n, ce, se), k, simplify)
    assert np.array_equal(grem, rem)
    assert np.array_equal(gcomp_of, comp_of)
    assert len(gcomps) == len(comps)
    for a, b in zip(gcomps, comps):
        assert np.array_equal(a, b)
    return len(rem), len(comps)


def test_random_graphs(ctx):
    rng = np.random.default_rng(61)
    say("device split, random graphs")
    for _ in range(300):
        n = int(rng.integers(1, 120))
        k = int(rng.integers(2, 6))
        e = random_graph(rng, n, float(rng.uniform(0.01, 0.25)))
        check(ctx, n, e, k, bool(rng.integers(0, 2)))


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_configs(ctx, cfg):
    import paper_2303_14335_amd as mp
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    say("device split, config", cfg, w.name)
    removed, ncomp = check(ctx, g.num_nodes, g.ce, w.k)
    assert ncomp > 0 and (removed > 0 or cfg == 3)   # config 3's 3-core is every node
    check(ctx, g.num_nodes, g.ce, w.k, simplify=False)


def test_deep_levels(ctx):
    say("device split, long paths and cycles")
    n = 3001   # path: peeled from both ends, one pair per level
    check(ctx, n, [(i, i + 1) for i in range(n - 1)], 2)
    n = 4000   # cycle: nothing removed at k = 2, one component, BFS depth n / 2
    assert check(ctx, n, [(i, (i + 1) % n) for i in range(n)], 2) == (0, 1)
    # a grid (4-regular inside): peeled from the corners inward at k = 4
    s = 60
    e = [(r * s + c, r * s + c + 1) for r in range(s) for c in range(s - 1)]
    e += [(r * s + c, (r + 1) * s + c) for r in range(s - 1) for c in range(s)]
    check(ctx, s * s, e, 4)
    check(ctx, s * s, e, 3)


def test_edge_cases(ctx):
    import paper_2303_14335_amd as mp
    say("device split, edge cases")
    assert check(ctx, 0, [], 3) == (0, 0)
    assert check(ctx, 1, [], 3) == (1, 0)
    assert check(ctx, 5, [], 2, simplify=False) == (0, 5)
    k4 = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    assert check(ctx, 4, k4, 4) == (4, 0)      # K4 at k = 4: all removed
    assert check(ctx, 4, k4, 3) == (0, 1)      # K4 at k = 3: the core
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_split_graph_device(ctx, mp.Graph(3, np.array([[0, 1]], np.int32),
                                                 np.zeros((0, 2), np.int32)), 1)
    assert e.value.code == -1
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_split_graph_device(ctx, mp.Graph(3, np.array([[0, 3]], np.int32),
                                                 np.zeros((0, 2), np.int32)), 3)
    assert e.value.code == -1
