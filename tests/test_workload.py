"""The seeded input generator (inputs only, shared by both sides)."""
import os

import numpy as np

import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    assert workload.splitmix64(1234567, len(vals)) == vals


def _touching_pairs(r):
    n = len(r)
    bad = 0
    for i in range(n):
        a = r[i]
        b = r[i + 1:]
        hit = (a[0] <= b[:, 2]) & (b[:, 0] <= a[2]) & (a[1] <= b[:, 3]) & (b[:, 1] <= a[3])
        bad += int(hit.sum())
    return bad


def test_generator_shapes_and_no_touching():
    r, skipped = workload.generate(2000, 12000, seed=3)
    assert skipped == 0 and len(r) == 2000
    w = r[:, 2] - r[:, 0]
    h = r[:, 3] - r[:, 1]
    short = np.minimum(w, h)
    long_ = np.maximum(w, h)
    assert np.all(short == 20)
    assert long_.min() >= 40 and long_.max() <= 200
    assert np.all(r[:, 0] >= 0) and np.all(r[:, 0] < 12000)
    assert np.all(r[:, 1] >= 0) and np.all(r[:, 1] < 12000)
    frac_h = float(np.mean(w > h))
    assert 0.45 < frac_h < 0.55
    assert _touching_pairs(r) == 0


def test_generator_deterministic_and_seeded():
    a, _ = workload.generate(500, 5000, seed=7)
    b, _ = workload.generate(500, 5000, seed=7)
    c, _ = workload.generate(500, 5000, seed=8)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_generator_skips_when_full():
    # a 100 nm window cannot hold 200 rectangles: most placements give up
    r, skipped = workload.generate(200, 100, seed=1, max_attempts=20)
    assert len(r) + skipped == 200 and skipped > 0
    assert _touching_pairs(r) == 0


def test_request_trace_statistics():
    t = workload.request_trace(0, 4000)
    gaps = np.diff(np.concatenate([[0.0], t["arrival_s"]]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 500) < 0.15 / 500
    n = t["n_rects"]
    assert n.min() >= 100 and n.max() <= 50000
    # log-uniform: the median sits near the geometric mean sqrt(100 * 50000)
    assert 1500 < np.median(n) < 3000
    side = t["side_nm"]
    assert np.allclose(side, np.round(3000 * np.sqrt(n / 300)), atol=1)
    assert len(set(t["seed"].tolist())) == 4000
