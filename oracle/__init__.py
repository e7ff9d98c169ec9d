"""ctypes binding of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's ``smoke()`` check
and the benchmark's CPU-baseline leg may import this module.  The product
library (``paper_2303_14335_amd``) never imports, links or calls it, and the
two share no code; they meet only on the seeded inputs from ``workload``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FEASIBLE, INFEASIBLE, BUDGET = 0, 1, 2
SIMPLIFY, MARK, STITCH, MINIMIZE = 1, 2, 4, 8
MINIMIZE_MAX_N = 64


class OrcComp(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("status", ctypes.c_int32),
                ("nodes", ctypes.c_int64), ("trace_hash", ctypes.c_uint64),
                ("depth_at_stop", ctypes.c_int32), ("stitches", ctypes.c_int32),
                ("first_node", ctypes.c_int32), ("num_edges", ctypes.c_int32),
                ("conflicts", ctypes.c_int32), ("min_nodes", ctypes.c_int32)]


def build() -> str:
    """Compile liboracle.so in place (plain C11, host only)."""
    src = os.path.join(_HERE, "oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                           "-fPIC", "-shared", "-pthread", "-o", tmp, src])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _p(t):
    return ctypes.POINTER(t)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; call oracle.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.orc_build_graph.restype = ctypes.c_int32
        lib.orc_build_graph.argtypes = [vp, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _p(ctypes.c_int32),
                                        _p(ctypes.c_int64), _p(vp),
                                        _p(ctypes.c_int64), _p(vp)]
        lib.orc_decompose.restype = ctypes.c_int32
        lib.orc_decompose.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                      ctypes.c_int64, vp, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, vp, vp,
                                      _p(ctypes.c_int32), _p(vp),
                                      _p(ctypes.c_int64), _p(ctypes.c_int64),
                                      _p(ctypes.c_int64)]
        lib.orc_solve_component.restype = ctypes.c_int32
        lib.orc_solve_component.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                            ctypes.c_int32, ctypes.c_int64, vp,
                                            _p(ctypes.c_int32),
                                            _p(ctypes.c_int64),
                                            _p(ctypes.c_uint64),
                                            _p(ctypes.c_int32)]
        lib.orc_solve_component_stitch.restype = ctypes.c_int32
        lib.orc_solve_component_stitch.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                                   ctypes.c_int32, ctypes.c_int64, vp, vp,
                                                   _p(ctypes.c_int32), _p(ctypes.c_int64),
                                                   _p(ctypes.c_uint64), _p(ctypes.c_int32)]
        lib.orc_mark_conflicts.restype = ctypes.c_int32
        lib.orc_mark_conflicts.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                           ctypes.c_int32, vp]
        lib.orc_minimize_component.restype = ctypes.c_int32
        lib.orc_minimize_component.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                               ctypes.c_int32, vp, ctypes.c_int64, vp,
                                               _p(ctypes.c_int64), _p(ctypes.c_int32),
                                               _p(ctypes.c_int32)]
        lib.orc_solve_many.restype = ctypes.c_int32
        lib.orc_solve_many.argtypes = [ctypes.c_int32, vp, vp, vp,
                                       ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                                       _p(ctypes.c_int64)]
        lib.orc_ec_matrix.restype = ctypes.c_int32
        lib.orc_ec_matrix.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                      ctypes.c_int32, _p(vp), _p(vp)]
        lib.orc_simplify.restype = ctypes.c_int32
        lib.orc_simplify.argtypes = [ctypes.c_int32, ctypes.c_int64, vp,
                                     ctypes.c_int32, ctypes.c_uint32, vp,
                                     _p(ctypes.c_int32), vp, vp, vp,
                                     _p(ctypes.c_int32)]
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [vp]
        _lib = lib
    return _lib


def _take(lib, ptr, count, dtype):
    if count == 0 or not ptr:
        if ptr:
            lib.orc_free(ptr)
        return np.zeros(0, dtype=dtype)
    buf = (ctypes.c_char * (count * np.dtype(dtype).itemsize)).from_address(ptr)
    arr = np.frombuffer(buf, dtype=dtype).copy()
    lib.orc_free(ptr)
    return arr


@dataclass
class Graph:
    num_nodes: int
    ce: np.ndarray   # int32 [m, 2], u < v, sorted
    se: np.ndarray   # int32 [s, 2]


def build_graph(rects: np.ndarray, dmin: int, split_len: int = 0) -> Graph:
    lib = _load()
    rects = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    nn = ctypes.c_int32()
    nce = ctypes.c_int64()
    nse = ctypes.c_int64()
    pce = ctypes.c_void_p()
    pse = ctypes.c_void_p()
    rc = lib.orc_build_graph(rects.ctypes.data, len(rects), dmin, split_len,
                             ctypes.byref(nn), ctypes.byref(nce),
                             ctypes.byref(pce), ctypes.byref(nse),
                             ctypes.byref(pse))
    if rc != 0:
        raise ValueError(f"orc_build_graph failed: {rc}")
    ce = _take(lib, pce.value, 2 * nce.value, np.int32).reshape(-1, 2)
    se = _take(lib, pse.value, 2 * nse.value, np.int32).reshape(-1, 2)
    return Graph(nn.value, ce, se)


@dataclass
class Decomposition:
    colors: np.ndarray       # int8 [num_nodes]
    comp_of: np.ndarray      # int32 [num_nodes]
    comps: np.ndarray        # structured records
    stitches: int
    conflicts: int
    uncolored: int


COMP_DTYPE = np.dtype([("size", np.int32), ("status", np.int32),
                       ("nodes", np.int64), ("trace_hash", np.uint64),
                       ("depth_at_stop", np.int32), ("stitches", np.int32),
                       ("first_node", np.int32), ("num_edges", np.int32),
                       ("conflicts", np.int32), ("min_nodes", np.int32)])


def decompose(g: Graph, k: int, budget: int, simplify: bool = True,
              mark: bool = False, stitch: bool = False, minimize: bool = False,
              min_budget: int = 10000) -> Decomposition:
    """Whole flow; mark=True colors the components left without a solution
    by the conflict-marking descent (mark_conflicts); stitch=True searches
    with the stitch-aware row order; minimize=True (implies mark) runs the
    Eq. 1 branch and bound (minimize_component, min_budget nodes) on every
    component of at most MINIMIZE_MAX_N nodes with a positive cost."""
    lib = _load()
    n = g.num_nodes
    ce = np.ascontiguousarray(g.ce, dtype=np.int32).reshape(-1, 2)
    se = np.ascontiguousarray(g.se, dtype=np.int32).reshape(-1, 2)
    colors = np.zeros(max(n, 1), dtype=np.int8)
    comp_of = np.zeros(max(n, 1), dtype=np.int32)
    nc = ctypes.c_int32()
    pcs = ctypes.c_void_p()
    st = ctypes.c_int64()
    cn = ctypes.c_int64()
    un = ctypes.c_int64()
    rc = lib.orc_decompose(n, len(ce), ce.ctypes.data, len(se), se.ctypes.data,
                           k, budget, min_budget,
                           (SIMPLIFY if simplify else 0) | (MARK if mark else 0)
                           | (STITCH if stitch else 0) | (MINIMIZE if minimize else 0),
                           colors.ctypes.data, comp_of.ctypes.data,
                           ctypes.byref(nc), ctypes.byref(pcs),
                           ctypes.byref(st), ctypes.byref(cn), ctypes.byref(un))
    if rc != 0:
        raise ValueError(f"orc_decompose failed: {rc}")
    raw = _take(lib, pcs.value, nc.value * COMP_DTYPE.itemsize, np.uint8)
    comps = raw.view(COMP_DTYPE) if nc.value else np.zeros(0, COMP_DTYPE)
    return Decomposition(colors[:n].copy(), comp_of[:n].copy(), comps,
                         st.value, cn.value, un.value)


@dataclass
class Solve:
    status: int
    nodes: int
    trace_hash: int
    depth_at_stop: int
    colors: np.ndarray


def solve_component(n: int, edges, k: int, budget: int, partner=None) -> Solve:
    """One component in local numbering; partner (n ints, -1 none) selects the
    stitch-aware row order."""
    lib = _load()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    colors = np.zeros(max(n, 1), dtype=np.int8)
    status = ctypes.c_int32()
    nodes = ctypes.c_int64()
    h = ctypes.c_uint64()
    d = ctypes.c_int32()
    part = None if partner is None else np.ascontiguousarray(np.asarray(partner, dtype=np.int32))
    rc = lib.orc_solve_component_stitch(n, len(e), e.ctypes.data, k, budget,
                                        None if part is None else part.ctypes.data,
                                        colors.ctypes.data, ctypes.byref(status),
                                        ctypes.byref(nodes), ctypes.byref(h),
                                        ctypes.byref(d))
    if rc != 0:
        raise ValueError(f"orc_solve_component failed: {rc}")
    return Solve(status.value, nodes.value, h.value, d.value, colors[:n].copy())


def mark_conflicts(n: int, edges, k: int) -> np.ndarray:
    """Conflict marking of Algorithm 1 on one component (local numbering):
    the no-backtracking descent whose empty columns take their last removed
    row.  Returns int8 colors, every node colored."""
    lib = _load()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    colors = np.zeros(max(n, 1), dtype=np.int8)
    rc = lib.orc_mark_conflicts(n, len(e), e.ctypes.data, k, colors.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_mark_conflicts failed: {rc}")
    return colors[:n].copy()


@dataclass
class Minimized:
    colors: np.ndarray
    nodes: int
    stopped: bool
    cost: int


def minimize_component(n: int, edges, k: int, colors, budget: int, partner=None) -> Minimized:
    """Eq. 1 branch and bound on one component from the complete incumbent
    `colors`; cost = 10 conflicts + stitches."""
    lib = _load()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    col = np.zeros(max(n, 1), dtype=np.int8)
    col[:n] = np.asarray(colors, dtype=np.int8)[:n]
    part = None if partner is None else np.ascontiguousarray(np.asarray(partner, dtype=np.int32))
    nodes = ctypes.c_int64()
    stopped = ctypes.c_int32()
    cost = ctypes.c_int32()
    rc = lib.orc_minimize_component(n, len(e), e.ctypes.data, k,
                                    None if part is None else part.ctypes.data, budget,
                                    col.ctypes.data, ctypes.byref(nodes), ctypes.byref(stopped),
                                    ctypes.byref(cost))
    if rc != 0:
        raise ValueError(f"orc_minimize_component failed: {rc}")
    return Minimized(col[:n].copy(), nodes.value, bool(stopped.value), cost.value)


def solve_many(sizes, edge_lists, k: int, budget: int, threads: int, passes: int = 1):
    """Components solved over `threads` host threads, the whole set repeated
    `passes` times in one call; returns a dict with the first pass's
    per-component status, nodes, trace_hash and concatenated local colors,
    and total_nodes over every pass."""
    lib = _load()
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    counts = np.array([len(e) for e in edge_lists], dtype=np.int64)
    edges = (np.ascontiguousarray(np.concatenate([np.asarray(e, np.int32).reshape(-1, 2)
                                                  for e in edge_lists]))
             if len(edge_lists) else np.zeros((0, 2), np.int32))
    cnt = len(sizes)
    colors = np.zeros(max(int(sizes.sum()), 1), dtype=np.int8)
    status = np.zeros(max(cnt, 1), dtype=np.int32)
    nodes = np.zeros(max(cnt, 1), dtype=np.int64)
    hashes = np.zeros(max(cnt, 1), dtype=np.uint64)
    total = ctypes.c_int64()
    rc = lib.orc_solve_many(cnt, sizes.ctypes.data, counts.ctypes.data,
                            edges.ctypes.data, k, budget, threads, passes,
                            colors.ctypes.data, status.ctypes.data,
                            nodes.ctypes.data, hashes.ctypes.data, ctypes.byref(total))
    if rc != 0:
        raise ValueError(f"orc_solve_many failed: {rc}")
    return {"status": status[:cnt], "nodes": nodes[:cnt],
            "trace_hash": hashes[:cnt], "colors": colors[:int(sizes.sum())],
            "total_nodes": total.value}


def ec_matrix(n: int, edges, k: int):
    """Dense 0/1 exact-cover matrix (rows n*k, cols n + m*k) for tests."""
    lib = _load()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    prp = ctypes.c_void_p()
    pci = ctypes.c_void_p()
    rc = lib.orc_ec_matrix(n, len(e), e.ctypes.data, k, ctypes.byref(prp),
                           ctypes.byref(pci))
    if rc != 0:
        raise ValueError(f"orc_ec_matrix failed: {rc}")
    rows = n * k
    rp = _take(lib, prp.value, rows + 1, np.int64)
    ci = _take(lib, pci.value, int(rp[-1]) if len(rp) else 0, np.int32)
    mat = np.zeros((rows, n + len(e) * k), dtype=np.uint8)
    for r in range(rows):
        mat[r, ci[rp[r]:rp[r + 1]]] = 1
    return mat


def simplify(g: Graph, k: int, simplify: bool = True):
    """Returns (removal_order, comp_of, [per-component global ids in local
    BFS order])."""
    lib = _load()
    n = g.num_nodes
    ce = np.ascontiguousarray(g.ce, dtype=np.int32).reshape(-1, 2)
    rem = np.zeros(max(n, 1), np.int32)
    comp_of = np.zeros(max(n, 1), np.int32)
    bfs = np.zeros(max(n, 1), np.int32)
    ptr = np.zeros(n + 2, np.int32)
    nrem = ctypes.c_int32()
    nc = ctypes.c_int32()
    rc = lib.orc_simplify(n, len(ce), ce.ctypes.data, k,
                          SIMPLIFY if simplify else 0, rem.ctypes.data,
                          ctypes.byref(nrem), comp_of.ctypes.data,
                          bfs.ctypes.data, ptr.ctypes.data, ctypes.byref(nc))
    if rc != 0:
        raise ValueError(f"orc_simplify failed: {rc}")
    comps = [bfs[ptr[c]:ptr[c + 1]].copy() for c in range(nc.value)]
    return rem[: nrem.value].copy(), comp_of[:n].copy(), comps
