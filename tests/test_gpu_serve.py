"""GPU tests of the continuous-batching server.

A request's result must be a function of its graph and options only: the
same alone (one-shot decomposition) as in a mix of concurrent requests,
for any per-tick slice of search nodes, with admission forced to wait by a
small device arena; an oversize request fails with MPLD_E_NOMEM instead of
waiting; traced requests keep their trace hash.
"""
import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.gpu

SIMPLIFY, TRACE = 1, 2


def say(*a):
    print("[case]", *a, flush=True)


def same(a, b):
    assert np.array_equal(a.colors, b.colors)
    assert np.array_equal(a.component_of, b.component_of)
    for f in a.components.dtype.names:
        assert np.array_equal(a.components[f], b.components[f]), f
    assert (a.stitches, a.conflicts, a.uncolored) == (b.stitches, b.conflicts, b.uncolored)


def check_oracle(got, req, budget, flags):
    """A served result against the oracle's own pipeline (its own graph
    builder, simplification, search, recovery) on the request's rectangles."""
    ref = oracle.decompose(oracle.build_graph(req["rects"], req["dmin"], req["split"]), req["k"],
                           budget, simplify=bool(flags & SIMPLIFY))
    assert np.array_equal(got.colors, ref.colors)
    assert np.array_equal(got.component_of, ref.comp_of)
    fields = ["size", "status", "nodes", "depth_at_stop", "stitches", "first_node", "num_edges"]
    if flags & TRACE:
        fields.append("trace_hash")
    for f in fields:
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert (got.stitches, got.conflicts, got.uncolored) == (ref.stitches, ref.conflicts,
                                                             ref.uncolored)


def requests(count, seed, n_max=6000, k=3, dmin=80, split=0):
    t = workload.request_trace(seed, count, n_min=100, n_max=n_max)
    out = []
    for i in range(count):
        rects, _ = workload.generate(int(t["n_rects"][i]), int(t["side_nm"][i]), int(t["seed"][i]))
        out.append(dict(rects=rects, dmin=dmin, split=split, k=k))
    return out


def alone(ctx, req, budget, flags):
    import paper_2303_14335_amd as mp
    g = mp.mpld_build_graph(req["rects"], req["dmin"], req["split"])
    return mp.mpld_decompose(ctx, g, req["k"], budget, flags)


@pytest.mark.parametrize("slice_nodes", [1, 7, 4096])
def test_mix_equals_alone(ctx, slice_nodes):
    import paper_2303_14335_amd as mp
    reqs = requests(40, seed=slice_nodes)
    say("serve mix, slice", slice_nodes, "requests", len(reqs))
    srv = mp.Server(ctx, slice_nodes=slice_nodes, max_components=4096, arena_bytes=32 << 20)
    tickets = [srv.submit_layout(r["rects"], r["dmin"], r["split"], r["k"], 10**6, SIMPLIFY | TRACE)
               for r in reqs]
    results = [srv.wait(t, 60_000_000) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for r, got in zip(reqs, results):
        assert got is not None
        same(got, alone(ctx, r, 10**6, SIMPLIFY | TRACE))
        check_oracle(got, r, 10**6, SIMPLIFY | TRACE)
        assert got.total_us >= got.queue_us >= 0


@pytest.mark.parametrize("simplify,builders,device_split",
                         [(True, 0, True), (False, 0, True), (True, 2, True), (True, 0, False),
                          (True, -1, True)])
def test_device_front_end_equals_alone(ctx, simplify, builders, device_split):
    # layouts of >= 4096 rects are built (and, with device_split, simplified
    # and split) on the device, by one builder or a pool of two; builders < 0
    # builds every graph on the host
    import paper_2303_14335_amd as mp
    reqs = requests(24, seed=31, n_max=12000)
    reqs += requests(4, seed=32, n_max=9000, k=4, split=120)
    flags = (SIMPLIFY if simplify else 0) | TRACE
    say("serve, simplify", simplify, "builders", builders, "device split", device_split,
        "requests", len(reqs))
    srv = mp.Server(ctx, slice_nodes=64, graph_builders=builders, device_split=device_split)
    tickets = [srv.submit_layout(r["rects"], r["dmin"], r["split"], r["k"], 20000, flags)
               for r in reqs]
    results = [srv.wait(t, 60_000_000) for t in tickets]
    srv.close()
    assert sum(len(r["rects"]) >= 4096 for r in reqs) >= 5
    for r, got in zip(reqs, results):
        same(got, alone(ctx, r, 20000, flags))
        check_oracle(got, r, 20000, flags)


def test_stitched_k4_heavy_components_sliced(ctx):
    import paper_2303_14335_amd as mp
    reqs = requests(12, seed=77, n_max=20000, k=4, dmin=120, split=120)
    say("serve k=4 stitched, slice 5")
    srv = mp.Server(ctx, slice_nodes=5, max_components=8192)
    tickets = [srv.submit_layout(r["rects"], r["dmin"], r["split"], r["k"], 20000, SIMPLIFY)
               for r in reqs]
    results = [srv.wait(t, 60_000_000) for t in tickets]
    ticks = srv.stats()["ticks"]
    srv.close()
    for r, got in zip(reqs, results):
        same(got, alone(ctx, r, 20000, SIMPLIFY))
        check_oracle(got, r, 20000, SIMPLIFY)
    assert ticks > 5   # heavy components took several ticks


def test_admission_waits_for_device_bytes(ctx):
    import paper_2303_14335_amd as mp
    # sixteen 2000-rectangle windows at the small workload's density: each
    # packed image is about 2 KB, so a 6 KB arena holds only a few of them,
    # and one-node slices keep every admitted request resident for many ticks
    reqs = []
    for i in range(16):
        rects, _ = workload.generate(2000, 7746, 1000 + i)
        reqs.append(dict(rects=rects, dmin=80, split=0, k=3))
    say("serve tiny arena")
    srv = mp.Server(ctx, arena_bytes=6 << 10, max_components=2048, slice_nodes=1)
    tickets = [srv.submit_layout(r["rects"], r["dmin"], r["split"], r["k"], 10**6) for r in reqs]
    results = [srv.wait(t, 60_000_000) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    assert st["admission_waits"] > 0
    assert st["peak_bytes"] <= 6 << 10
    for r, got in zip(reqs, results):
        same(got, alone(ctx, r, 10**6, SIMPLIFY))
        check_oracle(got, r, 10**6, SIMPLIFY)


def test_oversize_request_is_nomem_not_a_hang(ctx):
    import paper_2303_14335_amd as mp
    say("serve oversize")
    srv = mp.Server(ctx, arena_bytes=4096, max_components=64)
    rects, _ = workload.generate(20000, 8000, 3)
    t = srv.submit_layout(rects, 80, 0, 3, 1000)
    small, _ = workload.generate(50, 3000, 4)
    t2 = srv.submit_layout(small, 80, 0, 3, 1000)
    with pytest.raises(mp.MpldError) as e:
        srv.wait(t, 60_000_000)
    assert e.value.code == -2
    assert srv.wait(t2, 60_000_000) is not None     # later requests still run
    srv.close()


def test_bad_graph_and_unknown_ticket(ctx):
    import paper_2303_14335_amd as mp
    say("serve errors")
    srv = mp.Server(ctx)
    g = mp.Graph(3, np.array([[0, 5]]), np.zeros((0, 2), np.int32))
    t = srv.submit(g, 3, 100)
    with pytest.raises(mp.MpldError) as e:
        srv.wait(t, 60_000_000)
    assert e.value.code == -1
    with pytest.raises(mp.MpldError):
        srv.poll(123456789)
    srv.close()


def test_lds_tier_components_in_the_mix(ctx):
    import paper_2303_14335_amd as mp
    from algx_literal import random_graph
    rng = np.random.default_rng(8)
    graphs = []
    for n in (90, 150, 300):
        e = np.array(random_graph(rng, n, 5.0 / n), dtype=np.int32).reshape(-1, 2)
        graphs.append(mp.Graph(n, e, np.zeros((0, 2), np.int32)))
    say("serve LDS-tier components")
    srv = mp.Server(ctx, slice_nodes=11)
    tickets = [srv.submit(g, 3, 5000, SIMPLIFY | TRACE) for g in graphs]
    small = requests(6, seed=9)
    tickets += [srv.submit_layout(r["rects"], r["dmin"], 0, 3, 5000, SIMPLIFY | TRACE) for r in small]
    results = [srv.wait(t, 60_000_000) for t in tickets]
    srv.close()
    for g, got in zip(graphs, results[:3]):
        ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), 3, 5000)
        assert np.array_equal(got.colors, ref.colors)
        assert np.array_equal(got.components["nodes"], ref.comps["nodes"])
        assert np.array_equal(got.components["trace_hash"], ref.comps["trace_hash"])
    for r, got in zip(small, results[3:]):
        same(got, alone(ctx, r, 5000, SIMPLIFY | TRACE))
        check_oracle(got, dict(r, split=0, k=3), 5000, SIMPLIFY | TRACE)


def test_largest_serving_requests_vs_oracle(ctx):
    """The largest requests of the serving workload's own trace (10,000
    requests, seed 0; feature counts of at least 40,000, up to 50,000),
    served together with small ones at the serving options, each against
    the oracle's pipeline."""
    import paper_2303_14335_amd as mp
    from workload.configs import SERVE
    t = workload.request_trace(SERVE["seed"], SERVE["count"], rate=SERVE["rate"],
                               n_min=SERVE["n_min"], n_max=SERVE["n_max"],
                               base_side=SERVE["base_side"], base_n=SERVE["base_n"])
    big = [int(i) for i in np.flatnonzero(t["n_rects"] >= 40000)[:6]]
    small = [int(i) for i in np.flatnonzero(t["n_rects"] < 2000)[:10]]
    assert len(big) == 6
    reqs = []
    for i in big + small:
        rects, _ = workload.generate(int(t["n_rects"][i]), int(t["side_nm"][i]), int(t["seed"][i]))
        reqs.append(dict(rects=rects, dmin=SERVE["dmin_nm"], split=0, k=SERVE["k"]))
    say("serve the largest trace requests", big)
    srv = mp.Server(ctx)
    flags = SIMPLIFY | TRACE
    tickets = [srv.submit_layout(r["rects"], r["dmin"], r["split"], r["k"], SERVE["budget"], flags)
               for r in reqs]
    results = [srv.wait(tk, 60_000_000) for tk in tickets]
    srv.close()
    assert max(len(r["rects"]) for r in reqs) >= 40000
    for r, got in zip(reqs, results):
        check_oracle(got, r, SERVE["budget"], flags)


def test_heavy_lds_component_does_not_hold_up_small_requests(ctx):
    """A budget-heavy component above 64 nodes (about 0.35 s on the LDS
    tier) runs beside the ticks: small requests submitted after it finish
    long before it does, and every result equals the oracle's."""
    import time

    import paper_2303_14335_amd as mp
    n, deg, seed = 200, 5.6, 4   # INFEASIBLE after 501,238 search nodes (BFS numbering)
    e = np.asarray(workload.random_component(n, deg, seed), np.int32).reshape(-1, 2)
    heavy = mp.Graph(n, e, np.zeros((0, 2), np.int32))
    small = requests(20, seed=55, n_max=3000)
    say("serve a heavy LDS-tier component beside small requests")
    srv = mp.Server(ctx, slice_nodes=64)
    th = srv.submit(heavy, 3, 10**6, 0)
    time.sleep(0.03)
    ts = [srv.submit_layout(r["rects"], r["dmin"], 0, 3, 10**6, SIMPLIFY) for r in small]
    small_res = [srv.wait(t, 60_000_000) for t in ts]
    heavy_res = srv.wait(th, 60_000_000)
    srv.close()
    ref = oracle.decompose(oracle.Graph(n, e, np.zeros((0, 2), np.int32)), 3, 10**6,
                           simplify=False)
    for f in ("status", "nodes", "depth_at_stop"):
        assert np.array_equal(heavy_res.components[f], ref.comps[f]), f
    assert np.array_equal(heavy_res.colors, ref.colors)
    for r, got in zip(small, small_res):
        check_oracle(got, dict(r, split=0, k=3), 10**6, SIMPLIFY)
    slowest_small = max(g.total_us for g in small_res)
    assert heavy_res.total_us > 150_000
    assert slowest_small < heavy_res.total_us / 3, (slowest_small, heavy_res.total_us)


def test_conflict_marking_served(ctx):
    """MPLD_MARK_CONFLICTS in serving: register-tier components marked in
    the tick that ends their search, LDS-tier ones in their flight; every
    result equals the one-shot decomposition and the oracle's (marking on),
    for any slice."""
    import paper_2303_14335_amd as mp
    from algx_literal import random_graph
    MARK = 1 << 10
    rng = np.random.default_rng(12)
    graphs = []
    for n in (70, 120, 260):   # LDS tier, near the 3-colorability threshold
        e = np.array(random_graph(rng, n, 5.4 / n), dtype=np.int32).reshape(-1, 2)
        graphs.append(mp.Graph(n, e, np.zeros((0, 2), np.int32)))
    small = requests(16, seed=21, n_max=8000)
    for slice_nodes in (3, 4096):
        say("serve with conflict marking, slice", slice_nodes)
        srv = mp.Server(ctx, slice_nodes=slice_nodes)
        tg = [srv.submit(g, 3, 20000, SIMPLIFY | MARK) for g in graphs]
        ts = [srv.submit_layout(r["rects"], r["dmin"], 0, 3, 20000, SIMPLIFY | MARK | TRACE)
              for r in small]
        got_g = [srv.wait(t, 60_000_000) for t in tg]
        got_s = [srv.wait(t, 60_000_000) for t in ts]
        srv.close()
        for g, got in zip(graphs, got_g):
            same(got, mp.mpld_decompose(ctx, g, 3, 20000, SIMPLIFY | MARK))
            ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), 3, 20000, mark=True)
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "conflicts", "stitches"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
            assert got.uncolored == 0
        for r, got in zip(small, got_s):
            ref = oracle.decompose(oracle.build_graph(r["rects"], r["dmin"], 0), 3, 20000, mark=True)
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "trace_hash", "conflicts", "stitches"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
            assert (got.conflicts, got.uncolored) == (ref.conflicts, ref.uncolored)


def test_stitch_order_served(ctx):
    """MPLD_STITCH_ORDER in serving: stitch-ordered and plain requests in one
    server (separate tick launches), register-tier components resumed across
    ticks with their partner registers in the saved state (slice 3), and
    LDS-tier components with stitch pairs in the flights; every result
    equals the oracle's stitch-ordered decomposition."""
    import paper_2303_14335_amd as mp
    from algx_literal import random_graph
    STITCH = 1 << 11
    rng = np.random.default_rng(13)

    def stitched(count, n_lo, n_hi, k):
        ce, se, base = [], [], 0
        for _ in range(count):
            n = int(rng.integers(n_lo, n_hi + 1))
            e = random_graph(rng, n, min(0.95, float(rng.uniform(0.5, 1.4)) * 2.0 * k / n))
            adj = {tuple(x) for x in e} | {(b, a) for a, b in e}
            used = set()
            for _ in range(n):
                a, b = (int(x) for x in rng.integers(0, n, 2))
                if a != b and a not in used and b not in used and (a, b) not in adj:
                    used |= {a, b}
                    se.append((base + a, base + b))
            ce += [(base + a, base + b) for a, b in e]
            base += n
        return mp.Graph(base, np.array(ce, np.int32).reshape(-1, 2),
                        np.array(se, np.int32).reshape(-1, 2))

    graphs = [stitched(40, 4, 64, 3), stitched(6, 65, 300, 3), stitched(30, 4, 64, 4)]
    ks = [3, 3, 4]
    layouts = requests(6, seed=31, n_max=6000, split=120)
    for slice_nodes in (3, 4096):
        say("serve with the stitch-aware order, slice", slice_nodes)
        srv = mp.Server(ctx, slice_nodes=slice_nodes)
        tg = [srv.submit(g, k, 20000, STITCH | (TRACE if i % 2 else 0))
              for i, (g, k) in enumerate(zip(graphs, ks))]
        tp = [srv.submit(g, k, 20000, TRACE) for g, k in zip(graphs, ks)]   # plain order
        tl = [srv.submit_layout(r["rects"], r["dmin"], r["split"], 3, 20000,
                                SIMPLIFY | STITCH | TRACE) for r in layouts]
        got_g = [srv.wait(t, 60_000_000) for t in tg]
        got_p = [srv.wait(t, 60_000_000) for t in tp]
        got_l = [srv.wait(t, 60_000_000) for t in tl]
        srv.close()
        for i, (g, k, got) in enumerate(zip(graphs, ks, got_g)):
            ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), k, 20000,
                                   simplify=False, stitch=True)
            assert np.array_equal(got.colors, ref.colors)
            fields = ["status", "nodes", "depth_at_stop", "stitches"] + (["trace_hash"] if i % 2 else [])
            for f in fields:
                assert np.array_equal(got.components[f], ref.comps[f]), (f, i)
            assert got.stitches == ref.stitches
        for g, k, got in zip(graphs, ks, got_p):
            ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), k, 20000, simplify=False)
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "trace_hash", "stitches"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
        for r, got in zip(layouts, got_l):
            ref = oracle.decompose(oracle.build_graph(r["rects"], r["dmin"], r["split"]), 3, 20000,
                                   stitch=True)
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "trace_hash", "stitches", "depth_at_stop"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
            assert (got.stitches, got.uncolored) == (ref.stitches, ref.uncolored)


def test_minimize_served(ctx):
    """MPLD_MINIMIZE in serving: a register-tier component is marked and
    minimised for Eq. 1 by the wave that ends its search in a tick (its
    budget and node count per slot), LDS-tier components keep the marking's
    colors; with and without the stitch-aware order, at slices 3 and 4096,
    mixed with plain requests; every result equals the one-shot
    decomposition's and the oracle's (colors, node counts, minimisation
    counts, conflicts, stitches)."""
    import paper_2303_14335_amd as mp
    from algx_literal import random_graph
    MINIMIZE, STITCH = 1 << 13, 1 << 11
    rng = np.random.default_rng(17)

    def stitched(count, n_lo, n_hi, k, dens):
        ce, se, base = [], [], 0
        for _ in range(count):
            n = int(rng.integers(n_lo, n_hi + 1))
            e = random_graph(rng, n, min(0.95, float(rng.uniform(0.8, 1.6)) * dens * k / n))
            adj = {tuple(x) for x in e} | {(b, a) for a, b in e}
            used = set()
            for _ in range(n):
                a, b = (int(x) for x in rng.integers(0, n, 2))
                if a != b and a not in used and b not in used and (a, b) not in adj:
                    used |= {a, b}
                    se.append((base + a, base + b))
            ce += [(base + a, base + b) for a, b in e]
            base += n
        return mp.Graph(base, np.array(ce, np.int32).reshape(-1, 2),
                        np.array(se, np.int32).reshape(-1, 2))

    cases = [(stitched(40, 3, 40, 3, 2.0), 3, 0, 300), (stitched(20, 3, 64, 4, 2.2), 4, STITCH, 20000),
             (stitched(4, 65, 200, 3, 2.2), 3, 0, 50)]
    layouts = requests(4, seed=51, n_max=5000, dmin=100, split=120)
    for slice_nodes in (3, 4096):
        say("serve with the Eq. 1 minimisation, slice", slice_nodes)
        srv = mp.Server(ctx, slice_nodes=slice_nodes)
        tg = [srv.submit(g, k, 20000, MINIMIZE | extra, min_budget=mb) for g, k, extra, mb in cases]
        tp = [srv.submit(g, k, 20000, 0) for g, k, _, _ in cases]
        tl = [srv.submit_layout(r["rects"], r["dmin"], r["split"], 3, 20000,
                                SIMPLIFY | MINIMIZE | TRACE) for r in layouts]
        got_g = [srv.wait(t, 60_000_000) for t in tg]
        got_p = [srv.wait(t, 60_000_000) for t in tp]
        got_l = [srv.wait(t, 60_000_000) for t in tl]
        srv.close()
        for (g, k, extra, mb), got in zip(cases, got_g):
            same(got, mp.mpld_decompose(ctx, g, k, 20000, MINIMIZE | extra, min_budget=mb))
            ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), k, 20000, simplify=False,
                                   minimize=True, min_budget=mb, stitch=bool(extra & STITCH))
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "min_nodes", "conflicts", "stitches"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
            assert (got.conflicts, got.stitches, got.uncolored) == (ref.conflicts, ref.stitches,
                                                                     ref.uncolored)
        for (g, k, _, _), got in zip(cases, got_p):
            same(got, mp.mpld_decompose(ctx, g, k, 20000, 0))
        for r, got in zip(layouts, got_l):
            ref = oracle.decompose(oracle.build_graph(r["rects"], r["dmin"], r["split"]), 3, 20000,
                                   minimize=True)
            assert np.array_equal(got.colors, ref.colors)
            for f in ("status", "nodes", "trace_hash", "min_nodes", "conflicts", "stitches"):
                assert np.array_equal(got.components[f], ref.comps[f]), f
