"""The five synthetic workloads the solver is measured and checked on.

Each entry fixes the generator parameters (layoutgen.h), the minimum coloring
distance d_min (a conflict edge joins two features closer than d_min; the
paper uses 120 nm and 100 nm on its benchmarks, Sec. 3), the mask count k,
the optional stitch split length, and the per-component search-node budget.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    n_rects: int
    side_nm: int
    dmin_nm: int
    k: int
    split_len_nm: int  # 0 = no stitch split
    budget: int
    seed: int = 0


CONFIGS = {
    # 300 rectangles in a 3 um window, triple patterning, no stitches.
    0: Workload("small-k3", 300, 3000, 80, 3, 0, 1_000_000),
    # 200k rectangles in a 100 um window, triple patterning.
    1: Workload("200k-k3-d80", 200_000, 100_000, 80, 3, 0, 1_000_000),
    # 200k rectangles, quadruple patterning, d_min 120, midpoint stitch split
    # of every rectangle longer than 120 nm.
    2: Workload("200k-k4-d120-stitch", 200_000, 100_000, 120, 4, 120, 1_000_000),
    # 40k rectangles packed into a 12 um window (one giant component).
    3: Workload("40k-k3-d100-giant", 40_000, 12_000, 100, 3, 0, 10_000_000),
}

# Serving workload: 10,000 requests, Poisson arrivals at 500/s, feature count
# log-uniform in [100, 50000], window side scaled to keep config-0 density.
SERVE = dict(count=10_000, rate=500.0, n_min=100, n_max=50_000,
             base_side=3000, base_n=300, dmin_nm=80, k=3, budget=1_000_000,
             seed=0)
