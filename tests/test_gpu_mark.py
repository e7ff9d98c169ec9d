"""GPU parity of conflict marking (MPLD_MARK_CONFLICTS; Algorithm 1's
conflict candidates): components whose search ends INFEASIBLE or
BUDGET_EXHAUSTED are colored by the no-backtracking descent, bit-exactly as
the oracle's, on every tier; search records are unchanged; per-component
conflicts and stitches are counted on the colors.
"""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import complete, cycle, random_graph
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu

SIMPLIFY, TRACE, MARK = 1 << 0, 1 << 1, 1 << 10
FORCE = {"auto": 0, "lds": 1 << 4, "global": 1 << 5, "device": 1 << 7}
FIELDS = ("size", "status", "nodes", "trace_hash", "depth_at_stop", "stitches", "first_node",
          "num_edges", "conflicts")


def say(*a):
    print("[case]", *a, flush=True)


def compare(got, ref):
    assert np.array_equal(got.component_of, ref.comp_of)
    for f in FIELDS:
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)
    assert (got.stitches, got.conflicts, got.uncolored) == (ref.stitches, ref.conflicts,
                                                             ref.uncolored)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_marked_configs(ctx, cfg):
    import paper_2303_14335_amd as mp
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    say("marked config", cfg, w.name)
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget, mark=True)
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE | MARK)
    compare(got, ref)
    assert got.uncolored == 0 and got.conflicts > 0


def test_marked_config3_device_tier(ctx):
    import paper_2303_14335_amd as mp
    w = CONFIGS[3]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    say("marked config 3 on the device-wide tier")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget, mark=True)
    compare(mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | TRACE | MARK | FORCE["device"]), ref)


def _components(rng, k, count, n_lo, n_hi):
    comps = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi))
        p = min(0.95, float(rng.uniform(0.6, 1.8)) * 2.0 * k / max(n, 1))
        comps.append((n, random_graph(rng, n, p)))
    return comps


@pytest.mark.parametrize("tier", ["auto", "lds", "global", "device"])
@pytest.mark.parametrize("k", [2, 3, 4, 8])
def test_marked_components_every_tier(ctx, tier, k):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(700 + k)
    comps = [(k + 1, complete(k + 1)), (7, cycle(7)), (1, [])]
    if tier == "device":
        comps += _components(rng, k, 4, 65, 200)
    else:
        comps += _components(rng, k, 40, 1, 65 if tier == "auto" else 300)
    budget = 3000
    say("marked components, tier", tier, "k", k, "count", len(comps))
    recs, colors = mp.mpld_solve_components(ctx, comps, k, budget, FORCE[tier] | TRACE | MARK)
    failed = 0
    for (n, e), r, c in zip(comps, recs, colors):
        s = oracle.solve_component(n, e, k, budget)
        assert (int(r["status"]), int(r["nodes"]), int(r["trace_hash"])) == (s.status, s.nodes,
                                                                               s.trace_hash)
        want = s.colors if s.status == oracle.FEASIBLE else oracle.mark_conflicts(n, e, k)
        failed += s.status != oracle.FEASIBLE
        assert np.array_equal(c, want), (n, k, e)
        assert int(r["conflicts"]) == sum(1 for u, w in e if want[u] == want[w])
    assert failed > 0


def test_marked_budget_cut_components(ctx):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(91)
    comps = _components(rng, 3, 30, 20, 120)
    say("marked budget-cut components")
    for budget in (1, 5, 40):
        recs, colors = mp.mpld_solve_components(ctx, comps, 3, budget, MARK)
        for (n, e), r, c in zip(comps, recs, colors):
            s = oracle.solve_component(n, e, 3, budget)
            assert int(r["status"]) == s.status
            want = s.colors if s.status == oracle.FEASIBLE else oracle.mark_conflicts(n, e, 3)
            assert np.array_equal(c, want)


def test_batch_marks_on_every_solve(ctx):
    """A batch created with the flag marks on each solve, direct or replayed,
    and with the heavy-component engine."""
    import paper_2303_14335_amd as mp
    w = CONFIGS[2]
    rects, _ = workload.generate(40000, w.side_nm, w.seed)
    say("marked batch, 40k rects of config 2")
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), w.k, w.budget, mark=True)
    b = mp.Batch(ctx, g, w.k, w.budget, SIMPLIFY | MARK)
    for kw in (dict(direct=True), dict(direct=False), dict(direct=True, split=True)):
        b.solve(**kw)
        got = b.result()
        for f in ("status", "nodes", "stitches", "conflicts"):
            assert np.array_equal(got.components[f], ref.comps[f]), (kw, f)
        assert np.array_equal(got.colors, ref.colors), kw
    b.close()


def test_server_marks_conflicts(ctx):
    """A served request with MPLD_MARK_CONFLICTS (K4 and a 5-cycle with three
    masks: the clique is infeasible, so it is marked) equals the one-shot
    decomposition and the oracle's."""
    import paper_2303_14335_amd as mp
    say("server marks conflicts (K4 + C5)")
    edges = complete(4) + [(4 + a, 4 + b) for a, b in cycle(5)]
    g = mp.Graph(9, np.array(edges, dtype=np.int32), np.zeros((0, 2), np.int32))
    srv = mp.Server(ctx)
    got = srv.wait(srv.submit(g, 3, 100, SIMPLIFY | TRACE | MARK), 30_000_000)
    srv.close()
    ref = oracle.decompose(oracle.Graph(g.num_nodes, g.ce, g.se), 3, 100, mark=True)
    compare(got, ref)
    assert got.conflicts == 1 and got.uncolored == 0
