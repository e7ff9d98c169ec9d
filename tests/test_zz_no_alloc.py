"""The allocation-free entry point (mpld_solve_components_noalloc) against
mpld_solve_components through the C ABI: two calls in a row, the second
with a smaller input, records and colors bit for bit; its size limit and
unsupported flags are errors, not faults."""
import numpy as np
import pytest

from algx_literal import random_graph

pytestmark = pytest.mark.gpu

TRACE, MARK = 1 << 1, 1 << 10


def say(*a):
    print("[case]", *a, flush=True)


def batch(seed, count, n_hi, k):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(1, n_hi + 1))
        p = min(0.95, float(rng.uniform(0.5, 1.6)) * 2.0 * k / max(n, 1))
        out.append((n, random_graph(rng, n, p)))
    return out


def same(a, b):
    (ra, ca), (rb, cb) = a, b
    for f in ra.dtype.names:
        assert np.array_equal(ra[f], rb[f]), f
    assert len(ca) == len(cb)
    for x, y in zip(ca, cb):
        assert np.array_equal(x, y)


def test_noalloc_equals_solve_components_twice(ctx):
    import paper_2303_14335_amd as mp
    for k, flags in ((3, TRACE), (4, TRACE | MARK), (3, 0)):
        big = batch(100 + k, 400, 64, k)
        small = batch(200 + k, 37, 20, k)
        for name, comps in (("first, 400 components", big), ("second, 37 components", small)):
            say("noalloc", name, "k", k, "flags", flags)
            got = mp.mpld_solve_components_noalloc(ctx, comps, k, 20000, flags)
            ref = mp.mpld_solve_components(ctx, comps, k, 20000, flags)
            same(got, ref)


def test_noalloc_limits_are_errors(ctx):
    import paper_2303_14335_amd as mp
    say("noalloc limits")
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components_noalloc(ctx, [(65, [(0, 1)])], 3, 100)
    assert e.value.code == -7
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components_noalloc(ctx, [(4, [(0, 1)])], 3, 100, 1 << 13)
    assert e.value.code == -7
    # more items than the fixed scratch holds: 64-node components take 544 B
    # each, so 70,000 of them need about 38 MB of the 32 MiB
    many = [(64, [])] * 70000
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components_noalloc(ctx, many, 3, 100)
    assert e.value.code == -1
    with pytest.raises(mp.MpldError) as e:
        mp.mpld_solve_components_noalloc(ctx, [(3, [(0, 1), (1, 0)])], 3, 100)
    assert e.value.code == -1
    # still usable afterwards
    got = mp.mpld_solve_components_noalloc(ctx, [(4, [(0, 1), (1, 2), (2, 3), (0, 3)])], 3, 100)
    assert int(got[0]["status"][0]) == 0
    assert mp.mpld_solve_components_noalloc(ctx, [], 3, 100)[0].shape == (0,)
