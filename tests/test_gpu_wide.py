"""GPU parity of the big tier's two layouts against the oracle: one wave
with the planes and neighbour lists in LDS (level headers and undo log in
global memory), and a workgroup of waves sharing the column scan.  Cases:
components across the one-wave layout's range (2,049 to 16,384 nodes) and
just past it, small components forced onto the big tier, budget cuts
inside the search, a long infeasible search (hundreds of thousands of
backtracks through the global headers and log), the stitch-aware order,
subtree tasks and a served request.  Bit-exact: status, node count, trace
hash, depth at stop and colors of every component."""
import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.gpu

SIMPLIFY, TRACE = 1 << 0, 1 << 1
FORCE_GLOBAL = 1 << 5
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


def disjoint(parts):
    """One graph of disjoint components [(n, pairs)], ids offset in order."""
    ce, base = [], 0
    for n, e in parts:
        if len(e):
            ce.append(np.asarray(e, np.int64).reshape(-1, 2) + base)
        base += n
    ce = np.concatenate(ce).astype(np.int32) if ce else np.zeros((0, 2), np.int32)
    return base, ce


def batch_solve(ctx, g, k, budget, flags, one_wave, split=False):
    import paper_2303_14335_amd as mp
    b = mp.Batch(ctx, g, k, budget, flags)
    b.set_tune(big_one_wave=one_wave)
    b.solve(split=split)
    res = b.result()
    info = b.info()
    b.close()
    return res, info


@pytest.mark.parametrize("one_wave", [1, 0])
@pytest.mark.parametrize("k,deg,fits", [(3, 4.6, True), (2, 2.2, True), (4, 6.0, True),
                                        (4, 8.0, False), (5, 5.0, True), (6, 5.5, True),
                                        (7, 5.5, False)])
def test_big_components_vs_oracle(ctx, one_wave, k, deg, fits):
    """fits: every component takes the one-wave layout (at k = 4 and average
    degree 8 the 9000-node component's 144 KB of neighbour ids do not fit
    the workgroup's LDS, and k = 7 is past the layout's k, so those batches
    keep the workgroup layout)."""
    import paper_2303_14335_amd as mp
    parts = [(n, workload.random_component(n, deg, 40 + i))
             for i, n in enumerate((2049, 3000, 5200, 9000))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (20000, 777, 1):
        say("big components 2049-9000, k", k, "one wave", one_wave, "budget", budget)
        ref = oracle.decompose(og, k, budget, simplify=False)
        got, info = batch_solve(ctx, g, k, budget, TRACE, one_wave)
        assert info["num_global"] == 4
        assert (info["big_waves"] == 0) == bool(one_wave and fits)
        compare(got, ref)
        got, _ = batch_solve(ctx, g, k, budget, 0, one_wave)
        compare(got, ref, UNTRACED)


def test_one_wave_layout_limit(ctx):
    """16,384 nodes is the last size of the one-wave layout; a batch with a
    16,385-node component falls back to the workgroup."""
    import paper_2303_14335_amd as mp
    for n, wide in ((16384, True), (16385, False)):
        e = workload.random_component(n, 2.6, 7)
        g = mp.Graph(n, e, np.zeros((0, 2), np.int32))
        og = oracle.Graph(n, e, np.zeros((0, 2), np.int32))
        for budget in (30000, 40):
            say("one-wave layout limit, n", n, "budget", budget)
            ref = oracle.decompose(og, 3, budget, simplify=False)
            got, info = batch_solve(ctx, g, 3, budget, TRACE, 1)
            assert (info["big_waves"] == 0) == wide
            compare(got, ref)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_small_components_forced_big(ctx, k):
    import paper_2303_14335_amd as mp
    from algx_literal import random_graph
    rng = np.random.default_rng(7300 + k)
    parts = []
    for _ in range(80):
        n = int(rng.integers(1, 300))
        p = min(0.95, float(rng.uniform(0.5, 1.5)) * 2.0 * k / max(n, 1))
        parts.append((n, random_graph(rng, n, p)))
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (50000, 123, 2):
        ref = oracle.decompose(og, k, budget, simplify=False)
        for one_wave in (1, 0):
            say("small components forced onto the big tier, k", k, "budget", budget,
                "one wave", one_wave)
            got, info = batch_solve(ctx, g, k, budget, TRACE | FORCE_GLOBAL, one_wave)
            assert (info["big_waves"] == 0) == bool(one_wave)
            compare(got, ref)


@pytest.mark.parametrize("one_wave", [1, 0])
def test_long_infeasible_search(ctx, one_wave):
    """A 200-node component whose search visits every root row and ends
    INFEASIBLE after 501,238 nodes, forced onto the big tier: sequential and
    as root-row subtree tasks."""
    import paper_2303_14335_amd as mp
    n = 200
    e = workload.random_component(n, 5.6, 4)
    g = mp.Graph(n, e, np.zeros((0, 2), np.int32))
    ref = oracle.decompose(oracle.Graph(n, e, np.zeros((0, 2), np.int32)), 3, 10**6, simplify=False)
    assert int(ref.comps["nodes"][0]) == 501238
    for split in (False, True):
        say("long infeasible search, one wave", one_wave, "subtree tasks", split)
        got, _ = batch_solve(ctx, g, 3, 10**6, TRACE | FORCE_GLOBAL, one_wave, split=split)
        compare(got, ref)


def test_deep_backtracks_large_component(ctx):
    """A 2,500-node component near the 3-colorability threshold: backtracks
    of many levels, read back from the global headers and log."""
    import paper_2303_14335_amd as mp
    n = 2500
    e = workload.random_component(n, 4.9, 11)
    g = mp.Graph(n, e, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, e, np.zeros((0, 2), np.int32))
    for budget in (200000, 5001):
        say("deep backtracks, n 2500, budget", budget)
        ref = oracle.decompose(og, 3, budget, simplify=False)
        for one_wave in (1, 0):
            got, info = batch_solve(ctx, g, 3, budget, TRACE, one_wave)
            assert (info["big_waves"] == 0) == bool(one_wave)
            compare(got, ref)


@pytest.mark.parametrize("one_wave", [1, 0])
def test_feasible_after_backtracks(ctx, one_wave):
    """3,000-node components that reach a solution after a few hundred
    backtracking nodes (3,278 and 3,583 nodes): the colors come from the
    level headers in global memory."""
    import paper_2303_14335_amd as mp
    parts = [(3000, workload.random_component(3000, 3.8, 3)),
             (3000, workload.random_component(3000, 4.2, 1))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    ref = oracle.decompose(oracle.Graph(n, ce, np.zeros((0, 2), np.int32)), 3, 300000,
                           simplify=False)
    assert list(ref.comps["status"]) == [0, 0]
    assert sorted(int(x) for x in ref.comps["nodes"]) == [3278, 3583]
    say("feasible after backtracks, one wave", one_wave)
    got, _ = batch_solve(ctx, g, 3, 300000, TRACE, one_wave)
    compare(got, ref)


def stitched(rng, n, deg, seed):
    """A random component with stitch pairs between non-adjacent nodes."""
    e = workload.random_component(n, deg, seed)
    adj = {tuple(x) for x in e} | {(b, a) for a, b in e}
    se, used = [], set()
    for _ in range(n):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a != b and a not in used and b not in used and (a, b) not in adj:
            used |= {a, b}
            se.append((a, b))
    return e, np.array(se, np.int32).reshape(-1, 2)


@pytest.mark.parametrize("one_wave", [1, 0])
def test_stitch_order_big(ctx, one_wave):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(7700)
    ce, se, base = [], [], 0
    for i, n in enumerate((2100, 3500)):
        e, s = stitched(rng, n, 4.2, 60 + i)
        ce.append(e + base)
        se.append(s + base)
        base += n
    ce, se = np.concatenate(ce).astype(np.int32), np.concatenate(se).astype(np.int32)
    g = mp.Graph(base, ce, se)
    og = oracle.Graph(base, ce, se)
    for budget in (20000, 300):
        say("stitch order, big components, one wave", one_wave, "budget", budget)
        ref = oracle.decompose(og, 3, budget, simplify=False, stitch=True)
        got, info = batch_solve(ctx, g, 3, budget, STITCH | TRACE, one_wave)
        assert (info["big_waves"] == 0) == bool(one_wave)
        compare(got, ref)
        got, _ = batch_solve(ctx, g, 3, budget, STITCH, one_wave)
        compare(got, ref, UNTRACED)


def test_subtree_tasks_big(ctx):
    import paper_2303_14335_amd as mp
    parts = [(n, workload.random_component(n, 4.6, 90 + i)) for i, n in enumerate((2300, 4100))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (30000, 500):
        ref = oracle.decompose(og, 3, budget, simplify=False)
        for one_wave in (1, 0):
            say("subtree tasks, big components, one wave", one_wave, "budget", budget)
            got, _ = batch_solve(ctx, g, 3, budget, TRACE, one_wave, split=True)
            compare(got, ref)


def test_served_big_component(ctx):
    import paper_2303_14335_amd as mp
    parts = [(3000, workload.random_component(3000, 4.6, 5)), (40, workload.random_component(40, 3.0, 6))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    srv = mp.Server(ctx)
    try:
        for budget in (20000, 99):
            say("served request with a 3000-node component, budget", budget)
            ref = oracle.decompose(og, 3, budget, simplify=False)
            t = srv.submit(g, 3, budget, TRACE)
            compare(srv.wait(t, 120_000_000), ref)
    finally:
        srv.close()


def test_budget_sweep_big_layouts(ctx):
    """Budget cuts at every node count from 1 to 60 and a few larger ones
    on a 300-node component near the 3-colorability threshold, forced onto
    the big tier in both layouts: status, nodes, hash, depth at stop."""
    import paper_2303_14335_amd as mp
    n = 300
    e = workload.random_component(n, 5.0, 13)
    g = mp.Graph(n, e, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, e, np.zeros((0, 2), np.int32))
    say("budget sweep, both big-tier layouts, n 300")
    for budget in list(range(1, 61)) + [97, 1000, 4999, 65537]:
        ref = oracle.decompose(og, 3, budget, simplify=False)
        for one_wave in (1, 0):
            got, _ = batch_solve(ctx, g, 3, budget, TRACE | FORCE_GLOBAL, one_wave)
            compare(got, ref)


def test_one_wave_word_boundaries(ctx):
    """Sizes at the one-wave layout's word boundaries: 2,048 (one node word
    per lane, forced onto the big tier) and 2,049, 4,096 and 4,097, 8,192
    (a lane's keys in one 16-byte read) and 8,193 (in two)."""
    import paper_2303_14335_amd as mp
    parts = [(n, workload.random_component(n, 3.6, 70 + i))
             for i, n in enumerate((2048, 2049, 4096, 4097, 8192, 8193))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (12000, 2049, 5):
        say("one-wave word boundaries, budget", budget)
        ref = oracle.decompose(og, 3, budget, simplify=False)
        got, info = batch_solve(ctx, g, 3, budget, TRACE | FORCE_GLOBAL, 1)
        assert info["big_waves"] == 0 and info["num_global"] == 6
        compare(got, ref)


def test_mixed_big_layouts(ctx):
    """A batch whose big components take different layouts: 3,000 and 6,000
    nodes on one wave, 16,500 nodes (past the one-wave layout) on a
    workgroup; batched, as subtree tasks, and served."""
    import paper_2303_14335_amd as mp
    parts = [(3000, workload.random_component(3000, 4.6, 81)),
             (16500, workload.random_component(16500, 2.6, 82)),
             (6000, workload.random_component(6000, 4.6, 83))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (25000, 333):
        ref = oracle.decompose(og, 3, budget, simplify=False)
        for split in (False, True):
            say("mixed big-tier layouts, budget", budget, "subtree tasks", split)
            got, info = batch_solve(ctx, g, 3, budget, TRACE, 1, split=split)
            assert info["num_global"] == 3 and info["big_waves"] > 0
            compare(got, ref)
        srv = mp.Server(ctx)
        try:
            say("mixed big-tier layouts, served, budget", budget)
            compare(srv.wait(srv.submit(g, 3, budget, TRACE), 120_000_000), ref)
        finally:
            srv.close()


def test_autotune_tries_the_workgroup_layout(ctx, tmp_path):
    """A batch whose big components take the one-wave layout: the autotuner
    also times the workgroup layout (big_one_wave = 0) and must get the same
    records and colors from every candidate; the schedule it keeps goes to
    the cache with its big_one_wave."""
    import paper_2303_14335_amd as mp
    parts = [(n, workload.random_component(n, 4.6, 95 + i)) for i, n in enumerate((2500, 3500))]
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    ref = oracle.decompose(oracle.Graph(n, ce, np.zeros((0, 2), np.int32)), 3, 4000, simplify=False)
    say("autotune with one-wave big components")
    b = mp.Batch(ctx, g, 3, 4000, 0)
    cache = str(tmp_path / "tune.jsonl")
    t = b.autotune(reps=2, cache_path=cache)
    assert t["candidates"] >= 2
    b.solve()
    compare(b.result(), ref, UNTRACED)
    for one_wave in (0, 1):
        b.set_tune(big_one_wave=one_wave)
        assert (b.info()["big_waves"] == 0) == bool(one_wave)
        b.solve()
        compare(b.result(), ref, UNTRACED)
    b.close()
    with open(cache) as fh:
        assert '"big_one_wave": %d' % t["big_one_wave"] in fh.read()


@pytest.mark.parametrize("k", [3, 4])
def test_random_big_components(ctx, k):
    """Seeded random components of 2,049-12,000 nodes and average degree
    2.5-5.5, traced, at two budgets, on the default (per-component) big-tier
    layouts and on the workgroup layout alone."""
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(9100 + k)
    parts = []
    for i in range(8):
        n = int(rng.integers(2049, 12001))
        parts.append((n, workload.random_component(n, float(rng.uniform(2.5, 5.5)), 900 + 10 * k + i)))
    n, ce = disjoint(parts)
    g = mp.Graph(n, ce, np.zeros((0, 2), np.int32))
    og = oracle.Graph(n, ce, np.zeros((0, 2), np.int32))
    for budget in (3000, 137):
        ref = oracle.decompose(og, k, budget, simplify=False)
        for one_wave in (1, 0):
            say("random big components, k", k, "budget", budget, "one wave", one_wave)
            got, _ = batch_solve(ctx, g, k, budget, TRACE, one_wave)
            compare(got, ref)
