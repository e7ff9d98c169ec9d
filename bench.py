#!/usr/bin/env python3
"""Benchmark of the exact-cover layout decomposer on one MI355X.

A step is one pass of the whole device search over one batch: every
connected component of the simplified layout graph solved by Algorithm X
(min-count column, cover/uncover by bitset masks) in the tiered persistent
kernels, per-component results written to device memory.  The packed
exact-cover image is resident in HBM when the timed region starts (the host
front-end, packing and upload are timed separately and reported as
``frontend_ms`` / ``e2e_ms``).

The headline value is batched search nodes per second; the same JSON line
carries components/s, the plain one-component-per-launch solver on the same
batch, the dominant kernel's roofline and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("search nodes/s + components/s, batched vs plain on 1 GPU; "
          "p50/p99 layout latency")
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the register-tier kernel's sources and of its compile flags
    (include paths left out, as they differ between machines): the stored
    traffic counters belong to that kernel."""
    import importlib.util
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2303_14335_amd")
    for f in ("csrc/search_reg.hip", "csrc/reg_items.h", "csrc/wave_ops.h", "csrc/device_types.h",
              "csrc/trace.h", "csrc/min_core.h"):
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    spec = importlib.util.spec_from_file_location("_mpld_build_flags", os.path.join(pkg, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    flags, skip = [], False
    for x in mod.COMMON + mod.EXTRA.get("search_reg.hip", []):
        if skip:
            skip = False
        elif x == "-I":
            skip = True
        else:
            flags.append(x)
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


# Instruction issue per CU and cycle: the scalar unit takes one SALU
# instruction per cycle, and each of the four SIMDs one wave64 VALU
# instruction per four cycles; 256 CUs at 2.4 GHz.
CUS, CLOCK_HZ = 256, 2.4e9


def issue_fractions(pmc_sq_txt: str, kernel_ms: float):
    """SALU and VALU issue of reg_batched_kernel as fractions of the chip's
    issue rates, from the SQ counters of the committed rocprofv3 summary (per
    dispatch) over the live kernel duration; None without the summary."""
    if not os.path.exists(pmc_sq_txt):
        return None
    per = {}
    with open(pmc_sq_txt) as fh:
        for line in fh:
            if "reg_batched_kernel" not in line:
                continue
            for name in ("SQ_INSTS_SALU", "SQ_INSTS_VALU", "SQ_WAVES"):
                if f" {name} " in line:
                    per[name] = float(line.split()[-3])
    if len(per) < 3:
        return None
    cycles = kernel_ms * 1e-3 * CLOCK_HZ
    return {"salu_per_launch": per["SQ_INSTS_SALU"], "valu_per_launch": per["SQ_INSTS_VALU"],
            "waves": per["SQ_WAVES"],
            "salu_frac": per["SQ_INSTS_SALU"] / (cycles * CUS),
            "valu_frac": per["SQ_INSTS_VALU"] / (cycles * CUS),
            "source": os.path.relpath(pmc_sq_txt, ROOT)}


def oracle_components(rects, w):
    """Components of the oracle's own front-end as local edge lists."""
    import numpy as np
    import oracle
    g = oracle.build_graph(rects, w.dmin_nm, w.split_len_nm)
    _, comp_of, comps = oracle.simplify(g, w.k)
    adj = [[] for _ in range(g.num_nodes)]
    for a, b in g.ce.tolist():
        if comp_of[a] >= 0 and comp_of[b] >= 0:
            adj[a].append(b)
            adj[b].append(a)
    sizes, edge_lists = [], []
    for c in comps:
        loc = {int(v): i for i, v in enumerate(c.tolist())}
        e = [(loc[v], loc[u]) for v in c.tolist() for u in adj[v] if loc[v] < loc.get(u, -1)]
        sizes.append(len(c))
        edge_lists.append(np.asarray(e, dtype=np.int32).reshape(-1, 2))
    return g, sizes, edge_lists


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _timed_passes(sizes, edge_lists, w, threads: int, seconds: float):
    """One call of the oracle's runner with as many whole passes over every
    component as fit in about `seconds` (sized from one untimed pass)."""
    import oracle
    t = time.perf_counter()
    first = oracle.solve_many(sizes, edge_lists, w.k, w.budget, threads=threads)
    one = max(time.perf_counter() - t, 1e-6)
    passes = max(1, min(1 << 20, int(seconds / one)))
    t0 = time.perf_counter()
    r = oracle.solve_many(sizes, edge_lists, w.k, w.budget, threads=threads, passes=passes)
    el = time.perf_counter() - t0
    return first, r, passes, el


def cpu_legs(rects, w, seconds: float, gpu_comps):
    """The oracle as it stands on a bounded sample of the workload: whole
    passes over every component in one call of its runner, (1) on one
    thread pinned to one core, (2) on every host core (threads alive across
    passes, components claimed in chunks).  Both must reproduce the GPU
    batch's per-component status and node counts."""
    import numpy as np
    _, sizes, edge_lists = oracle_components(rects, w)
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        first1, r1, p1, el1 = _timed_passes(sizes, edge_lists, w, 1, seconds)
    finally:
        os.sched_setaffinity(0, set(allowed))
    threads = len(allowed)
    firstn, rn, pn, eln = _timed_passes(sizes, edge_lists, w, threads, seconds / 2)
    per_pass = int(np.sum(first1["nodes"]))
    agree = bool(np.array_equal(first1["status"], gpu_comps["status"])
                 and np.array_equal(first1["nodes"], gpu_comps["nodes"])
                 and np.array_equal(firstn["status"], first1["status"])
                 and np.array_equal(firstn["nodes"], first1["nodes"])
                 and r1["total_nodes"] == p1 * per_pass and rn["total_nodes"] == pn * per_pass)
    one = {"value": r1["total_nodes"] / el1, "unit": "search nodes/s", "cores": 1,
           "kind": "oracle",
           "sample": f"{p1} single-threaded pass(es) of the oracle's dancing-links search over "
                     f"all {len(sizes)} components of the workload ({per_pass} search nodes per "
                     f"pass) in one call, pinned to core {core}, {el1:.2f} s",
           "components_per_s": p1 * len(sizes) / el1,
           "agree": agree, "host": {"nproc": os.cpu_count(), "allowed_cores": threads,
                                    "cpu_model": _cpu_model()}}
    alln = {"value": rn["total_nodes"] / eln, "unit": "search nodes/s", "cores": threads,
            "kind": "oracle", "wall_ms_per_pass": 1000 * eln / pn,
            "cpu_model": _cpu_model(), "over_one_core": (rn["total_nodes"] / eln) /
            (r1["total_nodes"] / el1),
            "sample": f"{pn} pass(es) over all {len(sizes)} components on {threads} threads in "
                      f"one call, {eln:.2f} s", "agree": agree}
    return one, alln


def config_leg(mp, ctx, cfg: int, steps: int, split: bool):
    """Another workload as a device-resident batch: the host front-end, one
    untimed sequential solve as the reference, then `steps` back-to-back
    solves (with the heavy-component engine when `split`), whose status,
    node counts and colors must equal the reference's; plus the device
    solve time from image H2D to results D2H."""
    import numpy as np
    import torch

    import workload
    from workload.configs import CONFIGS
    w = CONFIGS[cfg]
    rects, skipped = workload.generate(w.n_rects, w.side_nm, w.seed)
    t0 = time.perf_counter()
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    t1 = time.perf_counter()
    b = mp.Batch(ctx, g, w.k, w.budget, mp.MPLD_SIMPLIFY)
    t2 = time.perf_counter()
    b.solve(direct=True)
    ref = b.result()
    rc = ref.components

    def same(r):
        return bool(np.array_equal(r.components["status"], rc["status"])
                    and np.array_equal(r.components["nodes"], rc["nodes"])
                    and np.array_equal(r.colors, ref.colors))

    b.solve(direct=True, split=split)
    ok = same(b.result())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(steps):
        b.solve(direct=True, split=split, timed=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - ts
    ok = ok and same(b.result())
    b.solve(direct=True, split=split, roundtrip=True)
    torch.cuda.synchronize()
    info = b.info()
    ok = ok and same(b.result())
    b.close()
    nodes = int(rc["nodes"].sum())
    return {"workload": f"config {cfg}: {w.name} ({w.n_rects} rectangles, "
                        f"{w.side_nm // 1000} um window, d_min {w.dmin_nm} nm, k={w.k}, "
                        f"split {w.split_len_nm} nm, budget {w.budget}, seed {w.seed})",
            "placed": int(len(rects)), "skipped": int(skipped), "layout_nodes": g.num_nodes,
            "conflict_edges": int(len(g.ce)), "components": len(rc),
            "max_component": int(rc["size"].max()) if len(rc) else 0,
            "tiers": {"wave": info["num_wave"], "lds": info["num_lds"],
                      "global": info["num_global"], "device": info["num_device"]},
            "search_nodes_per_step": nodes, "steps": steps, "heavy_engine": split,
            "ms_per_step": 1000 * wall / steps, "search_nodes_per_s": nodes * steps / wall,
            "components_per_s": len(rc) * steps / wall,
            "device_solve_ms": info["last_roundtrip_ms"],
            "statuses": {"feasible": int(np.sum(rc["status"] == 0)),
                         "infeasible": int(np.sum(rc["status"] == 1)),
                         "budget": int(np.sum(rc["status"] == 2))},
            "frontend_ms": {"graph": 1000 * (t1 - t0), "simplify_pack_upload": 1000 * (t2 - t1)},
            "same_as_sequential": ok}


def serve_leg(mp, ctx, count: int, seed: int, graph_builders: int = 0,
              device_split: bool = True):
    """Serving workload: `count` layout requests with Poisson arrivals at the
    configured rate, feature counts log-uniform in [100, 50000], window side
    scaled to the small workload's density; each is decomposed through the
    continuous-batching server.  Latency = finished result - arrival."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import workload
    from workload.configs import SERVE
    t = workload.request_trace(seed, count, rate=SERVE["rate"], n_min=SERVE["n_min"],
                               n_max=SERVE["n_max"], base_side=SERVE["base_side"],
                               base_n=SERVE["base_n"])

    def gen(i):
        return workload.generate(int(t["n_rects"][i]), int(t["side_nm"][i]), int(t["seed"][i]))[0]

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        rects = list(ex.map(gen, range(count)))
    srv = mp.Server(ctx, graph_builders=graph_builders, device_split=device_split)
    lags = np.zeros(count)
    tickets = []
    start = time.perf_counter()
    for i in range(count):
        target = start + float(t["arrival_s"][i])
        now = time.perf_counter()
        if target > now:
            time.sleep(target - now)
        lags[i] = max(0.0, time.perf_counter() - target)
        tickets.append(srv.submit_layout(rects[i], SERVE["dmin_nm"], 0, SERVE["k"], SERVE["budget"]))
    lat = np.zeros(count)
    queue = np.zeros(count)
    nodes = 0
    for i, tk in enumerate(tickets):
        r = srv.wait(tk)
        lat[i] = lags[i] * 1e6 + r.total_us
        queue[i] = r.queue_us
        nodes += int(r.components["nodes"].sum())
    end = time.perf_counter()
    st = srv.stats()
    srv.close()
    feats = int(np.sum(t["n_rects"]))
    return {"requests": count, "rate_per_s": SERVE["rate"], "seed": seed,
            "p50_ms": float(np.percentile(lat, 50)) / 1e3,
            "p99_ms": float(np.percentile(lat, 99)) / 1e3,
            "mean_ms": float(lat.mean()) / 1e3,
            "p99_queue_ms": float(np.percentile(queue, 99)) / 1e3,
            "max_client_lag_ms": float(lags.max()) * 1e3,
            "requests_per_s": count / (end - start),
            "features_per_s": feats / (end - start),
            "search_nodes_per_s": nodes / (end - start),
            "ticks": st["ticks"], "device_ms": st["device_ms"],
            "admission_waits": st["admission_waits"], "peak_device_bytes": st["peak_bytes"]}


def split_leg(mp, ctx, reps=5):
    """Device simplification and sub-graph split (mpld_split_graph_device,
    host validation, upload, kernels and download included) on a 50k-rect
    request at the serving density and on config 1's graph; best of `reps`."""
    import math

    import workload
    from workload.configs import CONFIGS, SERVE
    out = {}
    n = SERVE["n_max"]
    side = round(SERVE["base_side"] * math.sqrt(n / SERVE["base_n"]))
    cases = [(f"request {n} rects", workload.generate(n, side, 7)[0], SERVE["dmin_nm"], 0,
              SERVE["k"])]
    w = CONFIGS[1]
    cases.append((w.name, workload.generate(w.n_rects, w.side_nm, w.seed)[0], w.dmin_nm,
                  w.split_len_nm, w.k))
    for name, rects, dmin, split, k in cases:
        g = mp.mpld_build_graph(rects, dmin, split)
        mp.mpld_split_graph_device(ctx, g, k)
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            rem, _, comps = mp.mpld_split_graph_device(ctx, g, k)
            ts.append(time.perf_counter() - t)
        out[name] = {"nodes": g.num_nodes, "removed": int(len(rem)), "components": len(comps),
                     "ms": round(1000 * min(ts), 3)}
    return out


# Per-node latency probes (labelled as probes, not workloads): one connected
# random component per tier, run to its node budget on a single wave (or
# the whole device), so launch and setup costs vanish in the per-node time.
# The instances were picked so that the search runs to the budget.
PROBES = [
    # name, n, k, average degree, seed, budget, tier flag name; the register
    # probes run on one wave (root split off) and measure the per-node chain,
    # "..._root_split" runs the same instance with the root split
    ("register_k3_n64", 64, 3, 4.4, 26, 200000, "MPLD_FORCE_WAVE"),
    ("register_k3_n64_root_split", 64, 3, 4.4, 26, 200000, "MPLD_FORCE_WAVE"),
    ("register_k4_n64", 64, 4, 8.4, 0, 200000, "MPLD_FORCE_WAVE"),
    ("lds_small_k3_n1000", 1000, 3, 4.6, 0, 20000, "MPLD_FORCE_LDS"),
    ("lds_k3_n10000", 10000, 3, 4.6, 0, 20000, "MPLD_FORCE_GLOBAL"),
    # the same on the big tier's workgroup layout (lists in global memory)
    ("lds_k3_n10000_workgroup", 10000, 3, 4.6, 0, 20000, "MPLD_FORCE_GLOBAL"),
    ("lds_k3_n4000", 4000, 3, 4.6, 0, 20000, "MPLD_FORCE_GLOBAL"),
    ("lds_k3_n4000_workgroup", 4000, 3, 4.6, 0, 20000, "MPLD_FORCE_GLOBAL"),
    ("device_k3_n10000", 10000, 3, 4.6, 0, 2000, "MPLD_FORCE_DEVICE"),
    # an LDS-tier component whose search ends INFEASIBLE after visiting every
    # root row (501,238 nodes): sequential, and as root-row subtree tasks
    # ("..._split": the same exact counts), on the LDS and the big tier
    ("lds_k3_n200_infeasible", 200, 3, 5.6, 4, 1000000, "MPLD_FORCE_LDS"),
    ("lds_k3_n200_infeasible_split", 200, 3, 5.6, 4, 1000000, "MPLD_FORCE_LDS"),
    ("big_k3_n200_infeasible", 200, 3, 5.6, 4, 1000000, "MPLD_FORCE_GLOBAL"),
    ("big_k3_n200_infeasible_split", 200, 3, 5.6, 4, 1000000, "MPLD_FORCE_GLOBAL"),
]


def lds_rate(mp, ctx):
    """The chip's LDS read rate with ds_read_b64 and ds_read_b128 (every CU,
    no bank conflicts)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"cus": cus}
    for width in (8, 16):
        r = mp.mpld_measure_lds_read_rate(ctx, width, 2000)
        out[f"ds_read_b{8 * width}"] = {"GBps": round(r["GBps"], 1),
                                        "bytes_per_clock_per_cu": round(r["bytes_per_clock_per_cu"], 2)}
    out["peak_GBps"] = max(out["ds_read_b64"]["GBps"], out["ds_read_b128"]["GBps"])
    return out


def bitset_bytes_per_node(n: int, k: int, avg_degree: float) -> int:
    """Algorithmic bytes per search node of the bitset search: the k + 1
    planes of W = ceil(n / 64) words read by the count, 3 d_w words for the
    cover, the removed words kept and the uncover (d_w = min(W, mean degree
    rounded up)), 2 words of stack: 8 ((k + 1) W + 3 d_w + 2)."""
    import math
    w = (n + 63) // 64
    dw = min(w, max(1, math.ceil(avg_degree)))
    return 8 * ((k + 1) * w + 3 * dw + 2)


def latency_probe(mp, ctx, reps=3, names=None, lds=None):
    """lds: the measured LDS read rate (lds_rate()); the LDS-tier probes then
    carry their bitset bytes per node over their time as a fraction of one
    CU's share of it (a component runs on one CU)."""
    import numpy as np
    import torch
    import workload
    out = {}
    for name, n, k, deg, seed, budget, flag in PROBES:
        if names and name not in names:
            continue
        e = workload.random_component(n, deg, seed)
        g = mp.Graph(n, e, np.zeros((0, 2), np.int32))
        b = mp.Batch(ctx, g, k, budget, getattr(mp, flag))
        b.set_tune(root_split=1 if name.endswith("_root_split") else 0,
                   big_one_wave=0 if name.endswith("_workgroup") else 1)
        split = name.endswith("_split") and not name.endswith("_root_split")
        ms = []
        for _ in range(reps):
            b.solve(direct=True, split=split)
            torch.cuda.synchronize()
            ms.append(b.info()["last_search_ms"])
        nodes = int(b.result().components["nodes"].sum())
        b.close()
        out[name] = {"n": n, "k": k, "avg_degree": deg, "seed": seed, "nodes": nodes,
                     "ms": round(min(ms), 4), "ns_per_node": round(1e6 * min(ms) / max(nodes, 1), 2)}
        bpn = bitset_bytes_per_node(n, k, deg)
        gbps = bpn * nodes / (min(ms) * 1e-3) / 1e9
        out[name]["bitset_bytes_per_node"] = bpn
        out[name]["bitset_GBps"] = round(gbps, 3)
        if lds and flag != "MPLD_FORCE_WAVE":
            per_cu = lds["peak_GBps"] / lds["cus"]
            out[name]["lds_frac_of_one_cu"] = gbps / per_cu
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=1, help="workload (workload/configs.py)")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--split", action="store_true",
                    help="search heavy components as parallel subtrees (exact sequential counts)")
    ap.add_argument("--heavy-caps", type=str, default="",
                    help="with --split: first-pass cap,round cap[,levels] of the heavy engine")
    ap.add_argument("--launch", choices=["graph", "direct"], default="direct",
                    help="batched solve: replay the captured HIP graph or launch directly")
    ap.add_argument("--kernel-reps", type=int, default=50,
                    help="direct launches timed one by one for the kernel duration")
    ap.add_argument("--other-config-steps", type=int, default=20,
                    help="steps of the config 2 (heavy engine) and config 3 legs (0: skip)")
    ap.add_argument("--roundtrip-reps", type=int, default=20,
                    help="solves timed from image H2D to results D2H")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency-probe", action="store_true")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the per-tier latency probes and print them as one JSON line")
    ap.add_argument("--probes", type=str, default="",
                    help="comma-separated probe names to run (default: all)")
    ap.add_argument("--no-mark", action="store_true",
                    help="skip the conflict-marking leg (MPLD_MARK_CONFLICTS on the same workload)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="serving leg: requests of the serving workload (0 = skip)")
    ap.add_argument("--stitch-steps", type=int, default=20,
                    help="steps of the stitch-order leg on the stitch workload (0: skip)")
    ap.add_argument("--split-only", action="store_true",
                    help="only the device simplification/split leg (for profiling its kernels)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this size (counter scaling probe)")
    args = ap.parse_args()
    for name in ("plain_steps", "kernel_reps", "roundtrip_reps"):
        if getattr(args, name) < 1:
            ap.error(f"--{name.replace('_', '-')} must be at least 1")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "multi-GPU sharding of components is a design note only",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import numpy as np
    import torch

    import paper_2303_14335_amd as mp
    import workload
    from workload.configs import CONFIGS

    if args.split_only:
        ctx = mp.Context(0)
        out = {"device_split": split_leg(mp, ctx)}
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps(out), flush=True)
        return 0

    if args.probe_only:
        ctx = mp.Context(0)
        names = [x for x in args.probes.split(",") if x]
        lds = lds_rate(mp, ctx)
        out = {"lds_rate": lds, "latency_probe": latency_probe(mp, ctx, names=names, lds=lds)}
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps(out), flush=True)
        return 0

    w = CONFIGS[args.config]
    log(f"workload {w.name}: generating {w.n_rects} rectangles")
    rects, skipped = workload.generate(w.n_rects, w.side_nm, w.seed)

    ctx = mp.Context(0)
    stream = ctx.stream

    # ---- end to end once (front-end on the host, search on the device)
    t0 = time.perf_counter()
    g = mp.mpld_build_graph(rects, w.dmin_nm, w.split_len_nm)
    t1 = time.perf_counter()
    b = mp.Batch(ctx, g, w.k, w.budget, mp.MPLD_SIMPLIFY)
    if args.heavy_caps:
        caps = [int(x) for x in args.heavy_caps.split(",")]
        b.set_tune(heavy_first_cap=caps[0], heavy_round_cap=caps[1],
                   heavy_levels=caps[2] if len(caps) > 2 else 0)
    t2 = time.perf_counter()
    b.solve(split=args.split)
    res = b.result()
    t3 = time.perf_counter()
    # the first batch of a process also pays module loading and first
    # allocations: time a second creation of the same batch too
    tw = time.perf_counter()
    mp.Batch(ctx, g, w.k, w.budget, mp.MPLD_SIMPLIFY).close()
    warm_create_ms = 1000 * (time.perf_counter() - tw)
    info = b.info()
    comps = res.components
    total_nodes = int(comps["nodes"].sum())
    ncomp = len(comps)
    log(f"{g.num_nodes} nodes, {len(g.ce)} conflict edges, {ncomp} components, "
        f"{total_nodes} search nodes per pass")

    # ---- batched: K back-to-back solves (graph replays or direct launches)
    direct = args.launch == "direct"
    split = args.split
    for _ in range(args.warmup):
        b.solve(direct=direct, split=split, timed=False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ts = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        b.solve(direct=direct, split=split, timed=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - ts
    dev_ms = e0.elapsed_time(e1)
    ms_per_step = 1000.0 * wall / args.steps
    value = total_nodes * args.steps / wall
    log(f"batched: {ms_per_step:.4f} ms/step wall, {dev_ms / args.steps:.4f} ms/step device")

    # ---- the dominant kernel alone: direct launches, HIP events around it
    kms = []
    for _ in range(args.kernel_reps):
        b.solve(direct=True, split=split)
        torch.cuda.synchronize()
        kms.append(b.info()["last_search_ms"])
    single_ms = float(np.mean(kms))
    info_split = b.info()
    # the dominant kernel's duration: with one kernel launch per step (no
    # heavy engine) it is the timed region's device time per step, from the
    # HIP events recorded on the launch stream around the K steps; otherwise
    # the mean of the events around single solves
    one_kernel = info["launches"] == 1 and not split
    kernel_ms = dev_ms / args.steps if one_kernel else single_ms
    tune = b.get_tune()
    assert info["launches"] >= 1

    # ---- device solve time: the packed image copied from page-locked host
    # memory to the device, the search, records and colors copied back,
    # between two HIP events (MPLD_ROUNDTRIP); then the result is checked
    rts = []
    for _ in range(args.roundtrip_reps):
        b.solve(direct=True, split=split, roundtrip=True)
        torch.cuda.synchronize()
        rts.append(b.info()["last_roundtrip_ms"])
    res_rt = b.result()
    roundtrip = {"ms_median": float(np.median(rts)), "ms_min": float(np.min(rts)),
                 "reps": len(rts), "image_bytes": info["image_bytes"],
                 "search_nodes_per_s": total_nodes / (float(np.median(rts)) * 1e-3),
                 "same_result": bool(np.array_equal(res_rt.components["nodes"], comps["nodes"])
                                     and np.array_equal(res_rt.colors, res.colors))}
    log(f"device solve (H2D, search, D2H): {roundtrip['ms_median']:.4f} ms median")

    # ---- plain solver: one launch per component on the same batch
    b.solve(plain=True)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(args.plain_steps):
        b.solve(plain=True)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - tp
    plain_ms = 1000.0 * plain_wall / args.plain_steps
    res_plain = b.result()
    same = bool(np.array_equal(res_plain.components["nodes"], comps["nodes"])
                and np.array_equal(res_plain.colors, res.colors))
    log(f"plain: {plain_ms:.4f} ms/step")

    # ---- conflict marking (Algorithm 1's conflict candidates): the same
    # workload with MPLD_MARK_CONFLICTS, so that components left without a
    # solution are colored by the no-backtracking descent; a separate leg,
    # not the headline value
    mark = None
    if not args.no_mark:
        bm = mp.Batch(ctx, g, w.k, w.budget, mp.MPLD_SIMPLIFY | mp.MPLD_MARK_CONFLICTS)
        for _ in range(args.warmup):
            bm.solve(direct=direct, split=split, timed=False)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        for _ in range(args.steps):
            bm.solve(direct=direct, split=split, timed=False)
        torch.cuda.synchronize()
        mark_ms = 1000.0 * (time.perf_counter() - tm) / args.steps
        rm = bm.result()
        bm.close()
        failed = int(np.sum(rm.components["status"] != 0))
        mark = {"ms_per_step": mark_ms, "search_ms_per_step": ms_per_step,
                "marked_components": failed, "conflicts": int(rm.conflicts),
                "uncolored": int(rm.uncolored), "stitches": int(rm.stitches),
                "same_search": bool(np.array_equal(rm.components["nodes"], comps["nodes"]))}
        log(f"marking: {mark_ms:.4f} ms/step, {failed} components marked, {rm.conflicts} conflicts")

    # ---- stitch-aware row order (Eq. 1's stitch term) on the stitch
    # workload: the same batch searched in ascending row order and with
    # MPLD_STITCH_ORDER, both with the heavy-component engine (each checked
    # against its own sequential solve); a separate leg, not the headline
    stitch = None
    if args.stitch_steps:
        ws = next(c for c in CONFIGS.values() if c.split_len_nm > 0)
        rs, _ = workload.generate(ws.n_rects, ws.side_nm, ws.seed)
        gs = mp.mpld_build_graph(rs, ws.dmin_nm, ws.split_len_nm)
        legs = {}
        for name, fl in (("ascending", 0), ("stitch_order", mp.MPLD_STITCH_ORDER)):
            bs = mp.Batch(ctx, gs, ws.k, ws.budget, mp.MPLD_SIMPLIFY | fl)
            bs.solve(direct=True, timed=False)
            seq = bs.result()
            # untimed warm-up solves: after the plain leg's thousands of tiny
            # launches the first engine solves run measurably slower
            for _ in range(8):
                bs.solve(direct=direct, split=True, timed=False)
            torch.cuda.synchronize()
            tq = time.perf_counter()
            for _ in range(args.stitch_steps):
                bs.solve(direct=direct, split=True, timed=False)
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - tq) / args.stitch_steps
            rq = bs.result()
            cs = rq.components["stitches"]
            legs[name] = {"ms_per_step": ms,
                          "search_nodes": int(rq.components["nodes"].sum()),
                          "stitches": int(rq.stitches),
                          "stitches_in_searched_components": int(cs[cs >= 0].sum()),
                          "uncolored": int(rq.uncolored), "heavy_engine": True,
                          "same_as_sequential": bool(
                              np.array_equal(rq.colors, seq.colors)
                              and np.array_equal(rq.components["nodes"], seq.components["nodes"]))}
            bs.close()
        stitch = {"workload": ws.name, "steps": args.stitch_steps, **legs}
        log(f"stitch order: {legs['ascending']['stitches_in_searched_components']} -> "
            f"{legs['stitch_order']['stitches_in_searched_components']} stitches in searched "
            f"components, {legs['stitch_order']['ms_per_step']:.3f} ms/step")

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    # ---- roofline of the dominant kernel.  Algorithmic bytes per search
    # node of the bitset search: the k + 1 planes of W = ceil(n / 64) words
    # read by the count, 3 d_w words for the cover, the removed words kept
    # and the uncover (d_w = words that N(v) touches, min(W, mean degree)),
    # 2 words of stack push / pop: B_node = 8 ((k + 1) W + 3 d_w + 2); per
    # launch the sum over components of nodes x B_node.  The image bytes
    # (per component a 32 B descriptor, a 4 B queue entry and a 24 B record;
    # per node its neighbour mask or adjacency words and its 1 B color) are
    # reported beside it.
    def node_bytes(n, m):
        return bitset_bytes_per_node(n, w.k, 2 * m / max(n, 1))

    algo_bytes = int(sum(int(c["nodes"]) * node_bytes(int(c["size"]), int(c["num_edges"]))
                         for c in comps))
    image_bytes = (ncomp * (32 + 4 + 24) + info["core_nodes"] * 1
                   + 8 * int(np.sum(comps["size"][comps["size"] <= 64]))
                   + 4 * int(np.sum((comps["size"] + 2 + 2 * comps["num_edges"])[comps["size"] > 64])))
    achieved = algo_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = None
    issue = None
    prof = os.path.join(ROOT, "profiles", f"reg_batched_kernel_{w.name}_traffic.json")
    if os.path.exists(prof):
        with open(prof) as fh:
            t = json.load(fh)
        if t.get("kernel_source_hash") == kernel_source_hash():
            traffic = t.get("bytes_per_launch")
            issue = issue_fractions(os.path.join(ROOT, "profiles",
                                                 f"reg_batched_kernel_{w.name}_pmc_sq.txt"),
                                    kernel_ms)
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                "kernel": "reg_batched_kernel" if info["num_wave"] else "lds_batched_kernel",
                "kernel_us": round(kernel_ms * 1000.0, 3),
                "kernel_us_source": ("timed-region HIP events / steps" if one_kernel
                                     else "HIP events around single solves"),
                "single_solve_us": round(single_ms * 1000.0, 3),
                "issue": issue,
                "algorithmic_bytes_per_launch": algo_bytes,
                "bytes_per_search_node_w1": node_bytes(2, 1),
                "image_bytes_per_launch": image_bytes,
                "image_GBps": round(image_bytes / (kernel_ms * 1e-3) / 1e9, 3),
                "ns_per_search_node_per_wave": None}
    heavy = int(comps["nodes"].max()) if ncomp else 0
    if heavy:
        roofline["ns_per_search_node_per_wave"] = round(kernel_ms * 1e6 / heavy, 2)
    # the fixed cost of a launch inside the step: empty kernels launched back
    # to back (one workgroup of 256 lanes per component, and one wave)
    roofline["launch_floor_us"] = {
        "grid": max(1, ncomp), "block": 256,
        "us": round(mp.mpld_measure_launch_floor(ctx, max(1, ncomp), 256, 200), 3),
        "one_wave_us": round(mp.mpld_measure_launch_floor(ctx, 1, 64, 200), 3),
        # the same grid, every wave loading 64 B and storing 8 B: the floor
        # of a launch that touches device memory, as the search does
        "touch_us": round(mp.mpld_measure_touch_floor(ctx, max(1, ncomp), 256, 200), 3)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "search nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"config {args.config}: {w.name} ({w.n_rects} rectangles, "
                               f"{w.side_nm // 1000} um window, d_min {w.dmin_nm} nm, k={w.k}, "
                               f"split {w.split_len_nm} nm, budget {w.budget}, seed {w.seed})",
                   "components": ncomp, "core_nodes": info["core_nodes"],
                   "max_component": info["max_size"], "search_nodes_per_step": total_nodes,
                   "tiers": {"wave": info["num_wave"], "lds": info["num_lds"],
                             "global": info["num_global"]},
                   "placed": int(len(rects)), "skipped": int(skipped),
                   "layout_nodes": g.num_nodes, "conflict_edges": int(len(g.ce))},
        "components_per_s": ncomp * args.steps / wall,
        "device_ms_per_step": dev_ms / args.steps,
        "device_solve": roundtrip,
        "launch": args.launch,
        "split_heavy": args.split,
        "heavy_engine": ({"tune": {x: tune[x] for x in ("heavy_first_cap", "heavy_round_cap",
                                                         "heavy_levels")},
                          "components": info_split["heavy_components"],
                          "rounds": info_split["split_rounds"], "tasks": info_split["split_tasks"],
                          "reruns": info_split["split_reruns"]} if args.split else None),
        "plain": {"ms_per_step": plain_ms, "search_nodes_per_s": total_nodes / (plain_ms * 1e-3),
                  "components_per_s": ncomp / (plain_ms * 1e-3), "launches": ncomp,
                  "same_result": same},
        "batched_over_plain": plain_ms / ms_per_step,
        "mark_conflicts": mark,
        "stitch_order": stitch,
        "frontend_ms": {"graph": 1000 * (t1 - t0), "simplify_pack_upload": 1000 * (t2 - t1),
                        "simplify_pack_upload_warm": warm_create_ms},
        "e2e_ms": 1000 * (t3 - t0),
        "roofline": roofline,
        "statuses": {"feasible": int(np.sum(comps["status"] == 0)),
                     "infeasible": int(np.sum(comps["status"] == 1)),
                     "budget": int(np.sum(comps["status"] == 2))},
        "stitches": res.stitches, "uncolored": res.uncolored,
    }
    out["other_configs"] = {}
    for cfg, split_c in ((2, True), (3, False)):
        if cfg == args.config or not args.other_config_steps:
            continue
        log(f"config {cfg} leg")
        out["other_configs"][f"config {cfg}"] = config_leg(mp, ctx, cfg, args.other_config_steps,
                                                          split_c)
    log("device split leg")
    out["device_split"] = split_leg(mp, ctx)
    if not args.no_latency_probe:
        log("LDS read rate and latency probes")
        out["lds_rate"] = lds_rate(mp, ctx)
        out["latency_probe"] = latency_probe(mp, ctx, lds=out["lds_rate"])
    if args.serve_requests:
        log(f"serving leg: {args.serve_requests} requests")
        out["serving"] = serve_leg(mp, ctx, args.serve_requests, 0)
        out["p50_latency_ms"] = out["serving"]["p50_ms"]
        out["p99_latency_ms"] = out["serving"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"], out["cpu_all_cores"] = cpu_legs(rects, w, args.cpu_seconds, comps)
        if not out["cpu_baseline"]["agree"]:
            log("ERROR: the oracle's per-component status / node counts differ from the GPU batch")
            print(json.dumps(out), flush=True)
            return 1
    b.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
