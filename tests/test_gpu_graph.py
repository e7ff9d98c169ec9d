"""GPU layout-graph builder (mpld_build_graph_device) against the oracle's
graph: the same node count, conflict pairs (u < v, sorted) and stitch pairs,
on the workloads and on edge cases (empty, one feature, coincident and
degenerate boxes, negative and widely spread coordinates, splits)."""
import numpy as np
import pytest

import oracle
import workload
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def same_graph(ctx, rects, dmin, split):
    import paper_2303_14335_amd as mp
    got = mp.mpld_build_graph_device(ctx, rects, dmin, split)
    ref = oracle.build_graph(rects, dmin, split)
    assert got.num_nodes == ref.num_nodes
    assert np.array_equal(got.ce.reshape(-1, 2), ref.ce.reshape(-1, 2))
    assert np.array_equal(got.se.reshape(-1, 2), ref.se.reshape(-1, 2))
    return got


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_workload_graphs(ctx, cfg):
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    say("device graph, config", cfg, w.name)
    g = same_graph(ctx, rects, w.dmin_nm, w.split_len_nm)
    assert len(g.ce) > 0


@pytest.mark.parametrize("n,side,dmin,split", [(5000, 7746, 80, 0), (20000, 15000, 120, 120),
                                               (50000, 38730, 80, 0), (3000, 2000, 200, 60)])
def test_serving_sizes(ctx, n, side, dmin, split):
    rects, _ = workload.generate(n, side, 11)
    say("device graph", n, side, dmin, split)
    same_graph(ctx, rects, dmin, split)


def test_edge_cases(ctx):
    say("device graph edge cases")
    empty = np.zeros((0, 4), np.int32)
    same_graph(ctx, empty, 80, 0)
    same_graph(ctx, np.array([[0, 0, 20, 100]], np.int32), 80, 0)
    same_graph(ctx, np.array([[0, 0, 20, 300]], np.int32), 80, 120)      # one split feature
    rng = np.random.default_rng(3)
    # coincident, degenerate (zero width) and negative boxes, spread widely
    x = rng.integers(-2_000_000, 2_000_000, 3000)
    y = rng.integers(-2_000_000, 2_000_000, 3000)
    w = rng.integers(0, 200, 3000)
    h = rng.integers(0, 200, 3000)
    r = np.stack([x, y, x + w, y + h], 1).astype(np.int32)
    r = np.concatenate([r, r[:50], r[100:160] + 30]).astype(np.int32)
    same_graph(ctx, r, 80, 0)
    same_graph(ctx, r, 5000, 100)
    # a dense clump: many features per grid cell
    c = np.stack([rng.integers(0, 400, 2000), rng.integers(0, 400, 2000)], 1)
    r2 = np.concatenate([c, c + rng.integers(0, 60, (2000, 2))], 1).astype(np.int32)
    same_graph(ctx, r2, 30, 40)


def test_invalid_rectangle_rejected(ctx):
    import paper_2303_14335_amd as mp
    say("device graph rejects a bad box")
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_build_graph_device(ctx, np.array([[10, 0, 0, 5]], np.int32), 80, 0)
    assert e.value.code == -1
