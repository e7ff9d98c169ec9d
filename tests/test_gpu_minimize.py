"""GPU parity of the Eq. 1 minimisation (MPLD_MINIMIZE, register tier)
against the oracle's branch and bound: colors, per-component
branch-and-bound node counts (negated when the budget stopped it),
conflicts and stitches, bit for bit; the search's own fields unchanged."""
import numpy as np
import pytest

import oracle
import workload
from algx_literal import complete, cycle, random_graph
from workload.configs import CONFIGS

pytestmark = pytest.mark.gpu

SIMPLIFY, TRACE, MARK, MINIMIZE = 1, 2, 1 << 10, 1 << 13
FORCE_LDS = 1 << 4


def say(*a):
    print("[case]", *a, flush=True)


def compare(got, ref):
    assert np.array_equal(got.component_of, ref.comp_of)
    for f in ("size", "status", "nodes", "depth_at_stop", "stitches", "first_node", "num_edges",
              "conflicts", "min_nodes"):
        assert np.array_equal(got.components[f], ref.comps[f]), f
    assert np.array_equal(got.colors, ref.colors)
    assert (got.stitches, got.conflicts, got.uncolored) == (ref.stitches, ref.conflicts,
                                                             ref.uncolored)


def with_partners(rng, n, edges, frac):
    es = {(min(u, w), max(u, w)) for u, w in edges}
    se = []
    perm = rng.permutation(n)
    for i in range(0, n - 1, 2):
        a, b = int(perm[i]), int(perm[i + 1])
        if rng.random() < frac and (min(a, b), max(a, b)) not in es:
            se.append((min(a, b), max(a, b)))
    return np.asarray(se, np.int32).reshape(-1, 2)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_random_components_with_stitches(ctx, k):
    import paper_2303_14335_amd as mp
    rng = np.random.default_rng(500 + k)
    say("minimise random components, k", k)
    for it in range(40):
        n = int(rng.integers(2, 65))
        e = random_graph(rng, n, min(0.95, float(rng.uniform(0.8, 1.8)) * 2.0 * k / n))
        ce = np.asarray(e, np.int32).reshape(-1, 2)
        se = with_partners(rng, n, e, 0.5)
        g = mp.Graph(n, ce, se)
        for mb in (1, 7, 300, 20000):
            got = mp.mpld_decompose(ctx, g, k, 20000, MINIMIZE, min_budget=mb)
            ref = oracle.decompose(oracle.Graph(n, ce, se), k, 20000, simplify=False,
                                   minimize=True, min_budget=mb)
            compare(got, ref)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_configs_minimised(ctx, cfg):
    import paper_2303_14335_amd as mp
    w = CONFIGS[cfg]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    og = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    assert np.array_equal(g.ce, og.ce) and np.array_equal(g.se, og.se)
    say("minimise config", cfg)
    mb = 5000
    got = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | MINIMIZE, min_budget=mb)
    ref = oracle.decompose(og, w.k, w.budget, minimize=True, min_budget=mb)
    compare(got, ref)
    marked = mp.mpld_decompose(ctx, g, w.k, w.budget, SIMPLIFY | MARK)
    c_min = 10 * got.components["conflicts"] + got.components["stitches"]
    c_mark = 10 * marked.components["conflicts"] + marked.components["stitches"]
    assert np.all(c_min <= c_mark)
    assert got.conflicts <= marked.conflicts
    assert np.any(got.components["min_nodes"] != 0)


def test_batches_and_heavy_engine_keep_the_minimisation(ctx):
    """A batch solved several times, by direct launches, the captured graph
    and the heavy-component engine, gives the one-shot result."""
    import paper_2303_14335_amd as mp
    w = CONFIGS[2]
    rects, _ = workload.generate(60000, w.side_nm // 2, 5)
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    say("minimise in batches, 60k rects at config 2's settings")
    ref = oracle.decompose(oracle.build_graph(rects, w.dmin_nm, w.split_len_nm), w.k, 50000,
                           minimize=True, min_budget=2000)
    b = mp.Batch(ctx, g, w.k, 50000, SIMPLIFY | MINIMIZE, min_budget=2000)
    for how in ("direct", "graph", "split", "direct"):
        if how == "graph":
            b.set_tune(use_graph=1)
        b.solve(direct=how == "direct", split=how == "split")
        compare(b.result(), ref)
    b.close()


def test_solve_components_and_closed_forms(ctx):
    import paper_2303_14335_amd as mp
    say("minimise through mpld_solve_components")
    comps = [(5, complete(5)), (7, complete(7)), (4, complete(4)), (9, cycle(9)), (3, complete(3))]
    recs, cols = mp.mpld_solve_components(ctx, comps, 3, 1000, MINIMIZE, min_budget=100000)
    want = [20, 50, 10, 0, 0]   # Turan numbers x 10; C9 and K3 are 3-colorable
    for (n, e), r, c, wc in zip(comps, recs, cols, want):
        assert 10 * int(r["conflicts"]) == wc, (n, r)
        assert int(r["min_nodes"]) >= 0
        inc = oracle.solve_component(n, e, 3, 1000)
        start = inc.colors if inc.status == oracle.FEASIBLE else oracle.mark_conflicts(n, e, 3)
        m = oracle.minimize_component(n, e, 3, start, 100000)
        assert np.array_equal(c, m.colors)
        assert int(r["min_nodes"]) == (-m.nodes if m.stopped else m.nodes)


def test_unsupported_and_invalid(ctx):
    import paper_2303_14335_amd as mp
    say("minimise: forced LDS tier, negative budget")
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components(ctx, [(4, complete(4))], 3, 100, MINIMIZE | FORCE_LDS)
    assert e.value.code == -7
    g = mp.Graph(4, np.asarray(complete(4), np.int32), np.zeros((0, 2), np.int32))
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_decompose(ctx, g, 3, 100, MINIMIZE, min_budget=-1)
    assert e.value.code == -1
    srv = mp.Server(ctx)
    with pytest.raises(mp.MpldError) as e:
        srv.submit(g, 3, 100, MINIMIZE, min_budget=-1)
    assert e.value.code == -1
    srv.close()
