"""GPU parity of the stitch-aware row order (MPLD_STITCH_ORDER; Eq. 1 counts
a stitch for each pair of split halves colored differently): a chosen
column whose node's stitch partner is already colored on the path tries
that color's row first, the other rows ascending.  Status, node count, trace
hash, depth, colors and stitch counts equal the oracle's, traced and
untraced, with and without the root split of register-tier components.
"""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import random_graph
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu

SIMPLIFY, TRACE = 1 << 0, 1 << 1
FORCE_LDS, FORCE_GLOBAL, FORCE_DEVICE = 1 << 4, 1 << 5, 1 << 7
STITCH = 1 << 11
FIELDS = ("size", "status", "nodes", "trace_hash", "depth_at_stop", "stitches", "first_node",
          "num_edges")
UNTRACED = tuple(f for f in FIELDS if f != "trace_hash")


def say(*a):
    print("[case]", *a, flush=True)


def compare(got, ref, fields=FIELDS):
    assert np.array_equal(got.component_of, ref.comp_of)
    for f in fields:
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)
    assert (got.stitches, got.uncolored) == (ref.stitches, ref.uncolored)


def config_graph(cfg):
    import paper_2303_14335_amd as mp
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    return w, mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)


@pytest.mark.parametrize("trace", [True, False])
def test_stitch_config2(ctx, trace):
    import paper_2303_14335_amd as mp
    w, g = config_graph(2)
    say("stitch order, config 2, trace", trace)
    og = oracle.Graph(g.num_nodes, g.ce, g.se)
    ref = oracle.decompose(og, w.k, w.budget, stitch=True)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | STITCH | (TRACE if trace else 0))
    compare(got, ref, FIELDS if trace else UNTRACED)
    plain = oracle.decompose(og, w.k, w.budget)
    assert got.stitches < plain.stitches
    assert got.uncolored == plain.uncolored


@pytest.mark.parametrize("cfg", [0, 1])
def test_stitch_without_partners_is_plain(ctx, cfg):
    import paper_2303_14335_amd as mp
    w, g = config_graph(cfg)
    say("stitch order without stitch pairs, config", cfg)
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget)
    compare(mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE | STITCH), ref)


def random_layout(rng, k, count, n_lo, n_hi):
    """Disjoint random components of n_lo..n_hi nodes with random stitch
    pairs between non-adjacent nodes of the same component."""
    ce, se, base = [], [], 0
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        p = min(0.95, float(rng.uniform(0.4, 1.4)) * 2.0 * k / max(n, 1))
        e = random_graph(rng, n, p)
        adj = {tuple(x) for x in e} | {(b, a) for a, b in e}
        used = set()
        for _ in range(n):
            a, b = (int(x) for x in rng.integers(0, n, 2))
            if a != b and a not in used and b not in used and (a, b) not in adj:
                used |= {a, b}
                se.append((base + a, base + b))
        ce += [(base + a, base + b) for a, b in e]
        base += n
    ce = np.array(ce, np.int32).reshape(-1, 2)
    se = np.array(se, np.int32).reshape(-1, 2)
    return base, ce, se


@pytest.mark.parametrize("k", [2, 3, 4, 5])
@pytest.mark.parametrize("simplify", [True, False])
def test_stitch_random_layouts(ctx, k, simplify):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(5100 + 10 * k + simplify)
    n, ce, se = random_layout(rng, k, 150, 2, 64)
    g = mp.Graph(n, ce, se)
    og = oracle.Graph(n, ce, se)
    for budget in (20000, 40):
        say("stitch order, random layout, k", k, "simplify", simplify, "budget", budget)
        ref = oracle.decompose(og, k, budget, simplify=simplify, stitch=True)
        flags = (SIMPLIFY if simplify else 0) | STITCH
        compare(mp.mpld_decompose(ctx, g, k, budget, flags | TRACE), ref)
        compare(mp.mpld_decompose(ctx, g, k, budget, flags), ref, UNTRACED)


@pytest.mark.parametrize("root_split", [0, 1])
def test_stitch_batch_root_split(ctx, root_split):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(77 + root_split)
    n, ce, se = random_layout(rng, 3, 300, 4, 64)
    g = mp.Graph(n, ce, se)
    ref = oracle.decompose(oracle.Graph(n, ce, se), 3, 20000, simplify=False, stitch=True)
    say("stitch order, batch, root_split", root_split)
    b = mp.Batch(ctx, g, 3, 20000, STITCH)
    b.set_tune(root_split=root_split, root_split_min_n=4)
    for _ in range(2):   # replays keep the counter reset and the result
        b.solve()
        compare(b.result(), ref, UNTRACED)
    b.close()


def test_stitch_budget_cuts(ctx):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(41)
    n, ce, se = random_layout(rng, 3, 40, 8, 20)
    g = mp.Graph(n, ce, se)
    og = oracle.Graph(n, ce, se)
    say("stitch order, budget cuts")
    for budget in (1, 2, 3, 7, 15, 40, 120, 1000):
        ref = oracle.decompose(og, 3, budget, simplify=False, stitch=True)
        compare(mp.mpld_decompose(ctx, g, 3, budget, STITCH | TRACE), ref)
        compare(mp.mpld_decompose(ctx, g, 3, budget, STITCH), ref, UNTRACED)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_stitch_lds_and_big_tiers(ctx, k):
    """The stitch-aware order on the LDS and big tiers: components of 65-400
    nodes with stitch pairs (placed on the LDS tier, or forced onto the big
    tier), and small ones forced onto either; traced and untraced, at
    budgets that end inside the search and one that lets it finish."""
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(6100 + k)
    big_layout = random_layout(rng, k, 12, 65, 400)
    small_layout = random_layout(rng, k, 60, 2, 64)
    for name, (n, ce, se), extra in (("65-400 nodes", big_layout, 0),
                                     ("65-400 nodes, big tier", big_layout, FORCE_GLOBAL),
                                     ("small, LDS tier", small_layout, FORCE_LDS),
                                     ("small, big tier", small_layout, FORCE_GLOBAL)):
        g = mp.Graph(n, ce, se)
        og = oracle.Graph(n, ce, se)
        for budget in (30000, 300, 17):
            say("stitch order,", name, "k", k, "budget", budget)
            ref = oracle.decompose(og, k, budget, simplify=False, stitch=True)
            compare(mp.mpld_decompose(ctx, g, k, budget, STITCH | TRACE | extra), ref)
            compare(mp.mpld_decompose(ctx, g, k, budget, STITCH | extra), ref, UNTRACED)


def test_stitch_config3_big_tier(ctx):
    import paper_2303_14335_amd as mp
    w, g = config_graph(3)   # one component of about 40k nodes, big tier
    say("stitch order, config 3 on the big tier")
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget, stitch=True)
    compare(mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | STITCH | TRACE), ref)


def test_stitch_rejects_device_tier(ctx):
    import paper_2303_14335_amd as mp
    say("stitch order rejected on the device-wide tier")
    small = mp.Graph(3, np.array([[0, 1]], np.int32), np.zeros((0, 2), np.int32))
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_decompose(ctx, small, 3, 100, STITCH | FORCE_DEVICE)
    assert e.value.code == -7   # MPLD_E_UNSUPPORTED


def heavy_stitch_layout(rng, k, count, deg):
    """Components of 40-64 nodes near the colorability threshold (long
    searches) with random stitch pairs between non-adjacent nodes."""
    ce, se, base = [], [], 0
    for _ in range(count):
        n = int(rng.integers(40, 65))
        e = random_graph(rng, n, deg / n)
        adj = {tuple(x) for x in e} | {(b, a) for a, b in e}
        used = set()
        for _ in range(n):
            a, b = (int(x) for x in rng.integers(0, n, 2))
            if a != b and a not in used and b not in used and (a, b) not in adj:
                used |= {a, b}
                se.append((base + a, base + b))
        ce += [(base + a, base + b) for a, b in e]
        base += n
    return base, np.array(ce, np.int32).reshape(-1, 2), np.array(se, np.int32).reshape(-1, 2)


@pytest.mark.parametrize("k,deg,budget", [(3, 4.6, 300000), (4, 8.4, 300000), (3, 4.6, 20000)])
def test_stitch_with_heavy_engine(ctx, k, deg, budget):
    """The subtree engine under the stitch-aware order: tasks rebuild each
    path's row order and tried sets, so status, node count, depth and colors
    equal the sequential stitch-ordered search (budget cuts re-run
    sequentially); small caps force many rounds and deep splits."""
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(900 + 10 * k + (budget > 100000))
    n, ce, se = heavy_stitch_layout(rng, k, 30, deg)
    ref = oracle.decompose(oracle.Graph(n, ce, se), k, budget, simplify=False, stitch=True)
    assert int(ref.comps["nodes"].max()) > 1000
    g = mp.Graph(n, ce, se)
    say("stitch order with the heavy engine, k", k, "budget", budget)
    b = mp.Batch(ctx, g, k, budget, STITCH)
    for caps in ((64, 16, 0), (128, 256, 2), (256, 64, 1)):
        b.set_tune(heavy_first_cap=caps[0], heavy_round_cap=caps[1], heavy_levels=caps[2],
                   heavy_device=0)   # the host-driven setting still takes the device rounds
        b.solve(split=True)
        compare(b.result(), ref, UNTRACED)
    info = b.info()
    assert info["heavy_components"] > 0 and info["split_rounds"] >= 2
    b.close()


def test_stitch_config2_heavy_engine(ctx):
    import paper_2303_14335_amd as mp
    w, g = config_graph(2)
    say("stitch order, config 2, heavy engine")
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget, stitch=True)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY | STITCH)
    for _ in range(2):
        b.solve(split=True)
        compare(b.result(), ref, UNTRACED)
    assert b.info()["heavy_components"] > 0
    b.close()
