"""GPU parity: the HIP search (through the C ABI) against the oracle.

The bar is bit-exact: per component status, search-node count, trace hash,
depth at stop, colors; per node colors and component ids after recovery;
the Eq. 1 tallies.  Every case prints what names it before it runs.
"""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import complete, cycle, grotzsch, petersen, random_graph, wheel
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu

TRACE = 1 << 1
SIMPLIFY = 1 << 0
FORCE = {"wave": 1 << 3, "lds": 1 << 4, "global": 1 << 5, "device": 1 << 7}


def say(*a):
    print("[case]", *a, flush=True)


def compare_decomposition(got, ref):
    assert np.array_equal(got.component_of, ref.comp_of)
    rc = ref.comps
    gc = got.components
    assert len(gc) == len(rc)
    for f in ("size", "status", "nodes", "trace_hash", "depth_at_stop", "stitches",
              "first_node", "num_edges"):
        assert np.array_equal(gc[f], rc[f]), f
    assert np.array_equal(got.colors, ref.colors)
    assert (got.stitches, got.conflicts, got.uncolored) == (ref.stitches, ref.conflicts,
                                                             ref.uncolored)


def both_graphs(rects, w):
    """The product's layout graph and the oracle's own, built independently
    from the same rectangles; they must be equal."""
    import paper_2303_14335_amd as mp
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    og = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    assert g.num_nodes == og.num_nodes
    assert np.array_equal(g.ce, og.ce)
    assert np.array_equal(g.se, og.se)
    return g, og


def graph_of(cfg, n_rects=None):
    w = CONFIGS[cfg]
    rects, _ = workload.generate(n_rects or w.n_rects, w.side_nm, w.seed)
    return w, rects


@pytest.mark.parametrize("cfg", [0, 1])
def test_config_parity(ctx, cfg):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(cfg)
    say("config", cfg, w.name)
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE)
    compare_decomposition(got, ref)


def test_config2_parity_stitches(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2)
    say("config 2", w.name)
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE)
    compare_decomposition(got, ref)
    assert got.stitches > 0


def test_config3_giant_parity(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(3)
    say("config 3", w.name)
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE)
    compare_decomposition(got, ref)
    assert got.components["size"].max() > 30000


def solve_both(ctx, comps, k, budget, flags):
    import paper_2303_14335_amd as mp
    recs, colors = mp.mpld_solve_components(ctx, comps, k, budget, flags | TRACE)
    for (n, e), r, c in zip(comps, recs, colors):
        s = oracle.solve_component(n, e, k, budget)
        assert (int(r["status"]), int(r["nodes"]), int(r["trace_hash"]),
                int(r["depth_at_stop"])) == (s.status, s.nodes, s.trace_hash,
                                             s.depth_at_stop), (n, e, k, budget)
        assert np.array_equal(c, s.colors)


@pytest.mark.parametrize("tier", ["auto", "lds", "global", "device"])
def test_known_graphs_every_tier(ctx, tier):
    say("known graphs, tier", tier)
    flags = 0 if tier == "auto" else FORCE[tier]
    cases = [(4, complete(4), 3), (4, complete(4), 4), (5, complete(5), 4), (3, complete(3), 2),
             (7, cycle(7), 2), (8, cycle(8), 2), petersen() + (3,), grotzsch() + (3,),
             wheel(5) + (3,), wheel(6) + (3,), (1, [], 3), (0, [], 3)]
    for n, e, k in cases:
        solve_both(ctx, [(n, e)], k, 10**6, flags)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
def test_random_components_vs_oracle(ctx, k):
    rng = np.random.default_rng(1000 + k)
    comps = []
    for _ in range(300):
        n = int(rng.integers(1, 65))
        # near the k-colorability threshold so that the search backtracks
        p = min(0.95, float(rng.uniform(0.5, 1.6)) * 2.0 * k / max(n, 1))
        comps.append((n, random_graph(rng, n, p)))
    say("random components k", k, "count", len(comps))
    solve_both(ctx, comps, k, 20000, 0)


def test_lane_and_tier_boundaries(ctx):
    rng = np.random.default_rng(5)
    comps = []
    for n in (63, 64, 65, 127, 128, 129, 200):
        comps.append((n, random_graph(rng, n, 4.5 / n)))
        comps.append((n, cycle(n)))
    say("boundary sizes")
    for flags in (0, FORCE["lds"], FORCE["global"]):
        solve_both(ctx, comps, 3, 50000, flags)


def test_budget_sweep(ctx):
    rng = np.random.default_rng(9)
    comps = [(12, random_graph(rng, 12, 0.42)) for _ in range(6)]
    say("budget sweep")
    for b in list(range(1, 40)) + [100, 1000]:
        solve_both(ctx, comps, 3, b, 0)
        solve_both(ctx, comps, 3, b, FORCE["lds"])


def test_budget_sweep_device_tier(ctx):
    """Budget cuts on the device-wide tier (one cooperative launch per
    component): status, node count, hash and depth at every budget."""
    rng = np.random.default_rng(19)
    comps = [(int(n), random_graph(rng, int(n), 0.42)) for n in (9, 12, 14)]
    comps.append((90, random_graph(rng, 90, 4.6 / 90)))
    say("budget sweep, device-wide tier")
    for b in list(range(1, 25)) + [40, 100, 1000]:
        solve_both(ctx, comps, 3, b, FORCE["device"])


def test_larger_components_lds_tiers(ctx):
    rng = np.random.default_rng(21)
    comps = []
    for n in (80, 150, 300, 600, 1200):
        comps.append((n, random_graph(rng, n, 4.6 / n)))
    say("larger components")
    for flags in (0, FORCE["global"]):
        solve_both(ctx, comps, 3, 30000, flags)
    say("larger components, device-wide tier")
    solve_both(ctx, comps[:3], 3, 3000, FORCE["device"])


@pytest.mark.parametrize("k", [2, 4, 5, 8])
def test_lds_tiers_backtracking_every_k(ctx, k):
    """LDS and global tiers near the colorability threshold (deep
    backtracking, per-depth bit sets over several words), plus hub nodes of
    degree above 64 and 128 so that a cover takes several lane chunks."""
    rng = np.random.default_rng(2000 + k)
    comps = []
    for _ in range(24):
        n = int(rng.integers(1, 260))
        p = min(0.95, float(rng.uniform(0.6, 1.4)) * 2.0 * k / max(n, 1))
        comps.append((n, random_graph(rng, n, p)))
    for n, hub_deg in ((150, 70), (300, 140)):
        e = set(map(tuple, random_graph(rng, n, 1.5 * k / n)))
        for u in rng.choice(np.arange(1, n), size=hub_deg, replace=False):
            e.add((0, int(u)))
        comps.append((n, sorted(e)))
    say("LDS tiers, backtracking, k", k, "count", len(comps))
    for flags in (FORCE["lds"], FORCE["global"]):
        solve_both(ctx, comps, k, 20000, flags)


def test_config3_giant_device_tier(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(3)
    say("config 3 on the device-wide tier")
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE | FORCE["device"])
    compare_decomposition(got, ref)


def test_graph_replays_match_direct(ctx):
    """The captured HIP graph (schedule use_graph = 1), replayed several times
    with results read back in between, gives the direct launches' result."""
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2, 40000)
    say("graph replays, 40k rects of config 2")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    b = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY | TRACE)
    b.solve(direct=True)
    ref = b.result()
    b.set_tune(use_graph=1)
    for rep in range(4):
        b.solve()
        got = b.result()
        for f in ref.components.dtype.names:
            assert np.array_equal(got.components[f], ref.components[f]), (rep, f)
        assert np.array_equal(got.colors, ref.colors), rep
    b.close()


def test_plain_equals_batched_and_trace_off(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2, 40000)
    say("plain vs batched, 40k rects of config 2")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    b = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY | TRACE)
    b.solve(plain=False)
    r1 = b.result()
    b.solve(plain=True)
    r2 = b.result()
    b.close()
    for f in r1.components.dtype.names:
        assert np.array_equal(r1.components[f], r2.components[f]), f
    assert np.array_equal(r1.colors, r2.colors)
    b = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY)
    b.solve()
    r3 = b.result()
    b.solve()   # a replay of the same batch gives the same result
    r4 = b.result()
    b.close()
    for r in (r3, r4):
        assert np.array_equal(r.colors, r1.colors)
        assert np.array_equal(r.components["nodes"], r1.components["nodes"])
        assert np.array_equal(r.components["status"], r1.components["status"])


def test_simplify_off_isolated_nodes(ctx):
    import paper_2303_14335_amd as mp
    say("simplify off")
    g = mp.Graph(6, np.array([[0, 1], [1, 2], [0, 2]]), np.zeros((0, 2), np.int32))
    got = mp.mpld_decompose(ctx, g, 3, 1000, TRACE)
    ref = oracle.decompose(oracle.Graph(6, g.ce, g.se), 3, 1000, simplify=False)
    compare_decomposition(got, ref)
    g0 = mp.Graph(0, np.zeros((0, 2), np.int32), np.zeros((0, 2), np.int32))
    r0 = mp.mpld_decompose(ctx, g0, 3, 1000, SIMPLIFY)
    assert len(r0.colors) == 0 and len(r0.components) == 0


def test_invalid_arguments(ctx):
    import paper_2303_14335_amd as mp
    say("invalid arguments")
    g = mp.Graph(3, np.array([[0, 3]]), np.zeros((0, 2), np.int32))
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_decompose(ctx, g, 3, 10)
    assert e.value.code == -1
    g = mp.Graph(3, np.array([[0, 1]]), np.zeros((0, 2), np.int32))
    for k, budget in ((1, 10), (9, 10), (3, 0)):
        with pytest.raises(mp.MpldError) as e:
            mp.mpld_decompose(ctx, g, k, budget)
        assert e.value.code == -1
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components(ctx, [(70, cycle(70))], 3, 10, FORCE["wave"])
    assert e.value.code == -7


def test_product_validation_rejects_bad_graphs(ctx):
    """The library's own validation of a layout graph (no oracle involved):
    self loops, duplicate pairs in either orientation, a pair that is both a
    conflict and a stitch pair, a node in two stitch pairs, ids out of range
    and a negative node count are MPLD_E_INVALID, through the one-shot call,
    a batch and a server."""
    import paper_2303_14335_amd as mp
    say("product validation")
    z = np.zeros((0, 2), np.int32)
    bad = [
        mp.Graph(3, np.array([[1, 1]], np.int32), z),                       # self loop
        mp.Graph(3, np.array([[0, 1], [0, 1]], np.int32), z),               # duplicate
        mp.Graph(3, np.array([[0, 1], [1, 0]], np.int32), z),               # duplicate, reversed
        mp.Graph(4, np.array([[0, 1]], np.int32), np.array([[1, 0]], np.int32)),  # CE and SE
        mp.Graph(4, np.array([[0, 2]], np.int32), np.array([[0, 1], [0, 3]], np.int32)),  # two SE
        mp.Graph(4, np.array([[0, 2]], np.int32), np.array([[2, 2]], np.int32)),  # SE self loop
        mp.Graph(3, np.array([[0, -1]], np.int32), z),                      # negative id
        mp.Graph(3, np.array([[0, 1]], np.int32), np.array([[0, 3]], np.int32)),  # SE out of range
    ]
    for i, g in enumerate(bad):
        with pytest.raises(mp.MpldError) as e:
            mp.mpld_decompose(ctx, g, 3, 100, SIMPLIFY)
        assert e.value.code == -1, i
        with pytest.raises(mp.MpldError) as e:
            mp.Batch(ctx, g, 3, 100, SIMPLIFY)
        assert e.value.code == -1, i
    srv = mp.Server(ctx)
    for i, g in enumerate(bad):
        t = srv.submit(g, 3, 100)
        with pytest.raises(mp.MpldError) as e:
            srv.wait(t, 60_000_000)
        assert e.value.code == -1, i
    srv.close()
    # a valid graph still works after the rejections
    ok = mp.Graph(4, np.array([[0, 2], [1, 2]], np.int32), np.array([[0, 1]], np.int32))
    got = mp.mpld_decompose(ctx, ok, 3, 100, SIMPLIFY | TRACE)
    ref = oracle.decompose(oracle.Graph(4, ok.ce, ok.se), 3, 100)
    compare_decomposition(got, ref)


def test_roundtrip_solve_equals_plain_solve(ctx):
    """MPLD_ROUNDTRIP (image copied up from page-locked memory, search,
    results copied down, between events) gives the ordinary solve's result
    and a positive device solve time."""
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2, 40000)
    say("round-trip solve, 40k rects of config 2")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    b = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY | TRACE)
    b.solve(direct=True)
    ref = b.result()
    for rep in range(3):
        b.solve(direct=True, roundtrip=True)
        got = b.result()
        for f in ref.components.dtype.names:
            assert np.array_equal(got.components[f], ref.components[f]), (rep, f)
        assert np.array_equal(got.colors, ref.colors)
        assert b.info()["last_roundtrip_ms"] > 0
    b.set_tune(use_graph=1)
    b.solve(roundtrip=True)
    got = b.result()
    assert np.array_equal(got.colors, ref.colors)
    b.close()


def test_autotune_keeps_results_and_caches(ctx, tmp_path):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2, 30000)
    say("autotune on 30k rects of config 2")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    b = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY)
    b.solve()
    ref = b.result()
    cache = str(tmp_path / "tune.jsonl")
    t = b.autotune(reps=3, cache_path=cache)
    assert t["candidates"] > 1 and t["best_ms"] <= t["default_ms"] * 1.0001
    b.solve()
    got = b.result()
    assert np.array_equal(got.colors, ref.colors)
    assert np.array_equal(got.components["nodes"], ref.components["nodes"])
    # every schedule gives the same answer
    for wpb in (1, 2):
        for order in (0, 1):
            b.set_tune(waves_per_block=wpb, order=order, use_graph=0, max_blocks=64)
            b.solve()
            r = b.result()
            assert np.array_equal(r.colors, ref.colors)
            assert np.array_equal(r.components["status"], ref.components["status"])
    b.close()
    # a new batch of the same shape picks the cached schedule up
    import os
    os.environ["MPLD_TUNE_CACHE"] = cache
    try:
        b2 = mp.Batch(ctx, g, w.k, 20000, SIMPLIFY)
        t2 = b2.get_tune()
        b2.close()
    finally:
        del os.environ["MPLD_TUNE_CACHE"]
    assert t2["from_cache"] == 1
    assert (t2["waves_per_block"], t2["order"], t2["use_graph"]) == (
        t["waves_per_block"], t["order"], t["use_graph"])


def test_autotune_light_batch_root_split_candidates(ctx):
    # a light batch (config 1) also tries the root split's settings; every
    # candidate must reproduce the default's records and colors
    import paper_2303_14335_amd as mp
    w, rects = graph_of(1)
    say("autotune on config 1")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY)
    b.solve()
    ref = b.result()
    t = b.autotune(reps=3)
    assert t["candidates"] >= 6 and t["best_ms"] <= t["default_ms"] * 1.0001
    b.solve()
    got = b.result()
    assert np.array_equal(got.colors, ref.colors)
    assert np.array_equal(got.components["nodes"], ref.components["nodes"])
    b.close()


SPLIT = 1 << 8


def test_split_heavy_config2_matches_oracle(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2)
    say("config 2 with the heavy-component engine")
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | SPLIT)
    for f in ("size", "status", "nodes", "depth_at_stop", "stitches", "first_node"):
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)
    assert got.components["nodes"].max() > 100000   # a heavy component was split


@pytest.mark.parametrize("device_rounds", [0, 1])
def test_split_heavy_engines_agree(ctx, device_rounds):
    """Both heavy-component engines (rounds driven by the host, or chained on
    the device with the host resolving once) give the sequential result."""
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2)
    say("config 2, heavy engine with device rounds =", device_rounds)
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY)
    b.set_tune(heavy_device=device_rounds, heavy_first_cap=256, heavy_round_cap=128)
    for rep in range(2):
        b.solve(split=True)
        got = b.result()
        for f in ("status", "nodes", "depth_at_stop"):
            assert np.array_equal(got.components[f], ref.comps[f]), (f, rep)
        assert np.array_equal(got.colors, ref.colors), rep
    assert b.info()["split_rounds"] >= 3
    b.close()


def heavy_graphs(seed, count, n_lo, n_hi, deg):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append((n, random_graph(rng, n, deg / n)))
    return out


@pytest.mark.parametrize("k,deg,budget", [(3, 4.6, 300000), (4, 8.4, 300000), (3, 4.6, 20000)])
def test_split_heavy_random_components(ctx, k, deg, budget):
    import paper_2303_14335_amd as mp
    comps = heavy_graphs(k * 100 + int(deg), 40, 40, 64, deg)
    say("heavy random components k", k, "budget", budget)
    # the batch path: components through mpld_decompose with simplification off
    for n, e in comps:
        g = mp.Graph(n, np.asarray(e, np.int32).reshape(-1, 2), np.zeros((0, 2), np.int32))
        got = mp.mpld_decompose(ctx, g, k, budget, SPLIT)
        ref = oracle.decompose(oracle.Graph(n, g.ce, g.se), k, budget, simplify=False)
        for f in ("status", "nodes", "depth_at_stop"):
            assert np.array_equal(got.components[f], ref.comps[f]), (f, n, k, budget)
        assert np.array_equal(got.colors, ref.colors)


# ---- traced subtree engines: every subtree's trace hash appended in search
# order must give the sequential search's hash

@pytest.mark.parametrize("device_rounds", [0, 1])
def test_split_heavy_traced_matches_oracle(ctx, device_rounds):
    """Config 2 traced through the heavy-component engine with small caps
    (many rounds and split items), the hash included; traced batches always
    take the device-resident engine."""
    import paper_2303_14335_amd as mp
    w, rects = graph_of(2)
    say("config 2 traced, heavy engine, device rounds =", device_rounds)
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY | TRACE)
    b.set_tune(heavy_device=device_rounds, heavy_first_cap=256, heavy_round_cap=128)
    for rep in range(2):
        b.solve(split=True)
        got = b.result()
        for f in ("status", "nodes", "trace_hash", "depth_at_stop"):
            assert np.array_equal(got.components[f], ref.comps[f]), (f, rep)
        assert np.array_equal(got.colors, ref.colors), rep
    assert b.info()["split_rounds"] >= 3
    b.close()


@pytest.mark.parametrize("k,deg,budget", [(3, 4.6, 300000), (4, 8.4, 300000), (3, 4.6, 20000)])
def test_split_heavy_traced_random_components(ctx, k, deg, budget):
    import paper_2303_14335_amd as mp
    comps = heavy_graphs(k * 100 + int(deg) + 7, 30, 40, 64, deg)
    say("traced heavy random components k", k, "budget", budget)
    for n, e in comps:
        g = mp.Graph(n, np.asarray(e, np.int32).reshape(-1, 2), np.zeros((0, 2), np.int32))
        b = mp.Batch(ctx, g, k, budget, TRACE)
        b.set_tune(heavy_first_cap=64, heavy_round_cap=64)
        b.solve(split=True)
        got = b.result()
        b.close()
        ref = oracle.decompose(oracle.Graph(n, g.ce, g.se), k, budget, simplify=False)
        for f in ("status", "nodes", "trace_hash", "depth_at_stop"):
            assert np.array_equal(got.components[f], ref.comps[f]), (f, n, k, budget)
        assert np.array_equal(got.colors, ref.colors)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
def test_root_split_traced_random_components(ctx, k):
    """The root split with the trace hash (helpers' subtree hashes appended
    by the owner): a batch of random register-tier components, solved
    without the subtree engine (so every item of at least four nodes is
    root-split), at several budgets."""
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(5000 + k)
    edges, base = [], 0
    for _ in range(150):
        n = int(rng.integers(1, 65))
        p = min(0.95, float(rng.uniform(0.5, 1.6)) * 2.0 * k / max(n, 1))
        edges += [(a + base, b + base) for a, b in random_graph(rng, n, p)]
        base += n
    ce = np.asarray(edges, np.int32).reshape(-1, 2)
    g = mp.Graph(base, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(base, ce, np.zeros((0, 2), np.int32))
    say("root split traced, batch of random components, k", k)
    for budget in (20000, 1, 2, 3, 7, 40):
        ref = oracle.decompose(og, k, budget, simplify=False)
        b = mp.Batch(ctx, g, k, budget, TRACE)
        b.solve()
        got = b.result()
        b.close()
        for f in ("status", "nodes", "trace_hash", "depth_at_stop"):
            assert np.array_equal(got.components[f], ref.comps[f]), (f, budget)
        assert np.array_equal(got.colors, ref.colors), budget


# ---- untraced solves: the root split (helper waves searching the root's
# rows 1..3 of the largest register-tier components) must give the
# sequential status, node count, depth and colors

def solve_untraced(ctx, comps, k, budget):
    import paper_2303_14335_amd as mp
    recs, colors = mp.mpld_solve_components(ctx, comps, k, budget, 0)
    for (n, e), r, c in zip(comps, recs, colors):
        s = oracle.solve_component(n, e, k, budget)
        assert (int(r["status"]), int(r["nodes"]), int(r["depth_at_stop"])) == (
            s.status, s.nodes, s.depth_at_stop), (n, e, k, budget)
        assert np.array_equal(c, s.colors)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_config_parity_untraced(ctx, cfg):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(cfg)
    say("config", cfg, w.name, "untraced")
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY)
    for f in ("size", "status", "nodes", "depth_at_stop", "stitches", "first_node", "num_edges"):
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
def test_root_split_random_components(ctx, k):
    rng = np.random.default_rng(3000 + k)
    comps = []
    for _ in range(200):
        n = int(rng.integers(1, 65))
        p = min(0.95, float(rng.uniform(0.5, 1.6)) * 2.0 * k / max(n, 1))
        comps.append((n, random_graph(rng, n, p)))
    say("root split, random components, k", k)
    solve_untraced(ctx, comps, k, 20000)


def test_root_split_budget_cuts(ctx):
    rng = np.random.default_rng(31)
    comps = [(int(n), random_graph(rng, int(n), 0.4)) for n in rng.integers(8, 20, 40)]
    say("root split, budget cuts")
    for budget in (1, 2, 3, 7, 15, 40, 120, 1000):
        solve_untraced(ctx, comps, 3, budget)


# ---- subtree tasks of the LDS and big tiers (untraced solves): the k root
# rows searched in parallel, the sequential status, node count, depth and
# colors recomputed in row order

def solve_split_csr(ctx, comps, k, budget, flags):
    import paper_2303_14335_amd as mp
    recs, colors = mp.mpld_solve_components(ctx, comps, k, budget, flags)
    for (n, e), r, c in zip(comps, recs, colors):
        s = oracle.solve_component(n, e, k, budget)
        assert (int(r["status"]), int(r["nodes"]), int(r["depth_at_stop"])) == (
            s.status, s.nodes, s.depth_at_stop), (n, k, budget, flags)
        assert np.array_equal(c, s.colors)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_csr_subtree_tasks_random_components(ctx, k):
    rng = np.random.default_rng(4000 + k)
    comps = []
    for _ in range(30):
        n = int(rng.integers(65, 400))
        p = min(0.95, float(rng.uniform(0.6, 1.4)) * 2.0 * k / n)
        comps.append((n, random_graph(rng, n, p)))
    say("LDS/big-tier subtree tasks, random components, k", k)
    for flags in (0, FORCE["lds"], FORCE["global"]):
        solve_split_csr(ctx, comps, k, 30000, flags)


def test_csr_subtree_tasks_budget_cuts(ctx):
    """Budgets that end the search in row 0's subtree, exactly between two
    root rows, inside a later row's subtree (the re-run) and after every
    row."""
    rng = np.random.default_rng(4100)
    comps = [(int(n), random_graph(rng, int(n), 4.6 / int(n))) for n in (70, 90, 130, 200)]
    full = [oracle.solve_component(n, e, 3, 10**6) for n, e in comps]
    say("LDS/big-tier subtree tasks, budget cuts")
    budgets = {1, 2, 3, 5, 17, 100, 1000}
    for s in full:
        budgets |= {max(1, s.nodes - 1), s.nodes, s.nodes + 1}
    for flags in (FORCE["lds"], FORCE["global"]):
        for b in sorted(budgets):
            solve_split_csr(ctx, comps, 3, b, flags)


def test_csr_subtree_tasks_exact_boundaries(ctx):
    """Budget cuts at every node count where a root row's subtree ends, for
    components whose search visits several root rows."""
    rng = np.random.default_rng(4200)
    picked = []
    while len(picked) < 3:
        n = int(rng.integers(70, 120))
        e = random_graph(rng, n, 5.2 / n)
        s = oracle.solve_component(n, e, 3, 10**6)
        if s.status == oracle.INFEASIBLE and s.nodes > 20:
            picked.append((n, e, s.nodes))
    say("LDS/big-tier subtree tasks, every budget near the row boundaries")
    for n, e, total in picked:
        for b in range(1, min(total, 400) + 2):
            solve_split_csr(ctx, [(n, e)], 3, b, FORCE["lds"])


def test_csr_subtree_tasks_empty_and_tiny(ctx):
    """Components with no node (the root is the solution), one node and one
    edge on the forced LDS and big tiers, where every solve goes through the
    root-row subtree tasks, traced and untraced, at budgets 1..4."""
    comps = [(0, []), (1, []), (2, [(0, 1)]), (3, [(0, 1), (1, 2), (0, 2)])]
    say("LDS/big-tier subtree tasks, empty and tiny components")
    for flags in (FORCE["lds"], FORCE["global"]):
        for budget in (1, 2, 3, 4, 100):
            solve_split_csr(ctx, comps, 3, budget, flags)
            solve_both(ctx, comps, 3, budget, flags)


def test_csr_subtree_tasks_in_batches_and_config3(ctx):
    import paper_2303_14335_amd as mp
    w, rects = graph_of(3)
    say("config 3 untraced, subtree tasks on the big tier")
    g, og = both_graphs(rects, w)
    ref = oracle.decompose(og, w.k, w.budget)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY)
    for f in ("size", "status", "nodes", "depth_at_stop", "first_node", "num_edges"):
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY)
    for split in (False, True, True):
        b.solve(split=split)
        r = b.result()
        assert np.array_equal(r.components["nodes"], ref.comps["nodes"])
        assert np.array_equal(r.colors, ref.colors)
    assert b.info()["split_tasks"] >= 3
    b.close()
