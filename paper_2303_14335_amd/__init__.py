"""MI355X exact-cover multiple-patterning layout decomposer (Python binding).

Thin wrapper over the C ABI in ``include/mpld.h``: every function here only
marshals arguments; every step of the decomposition runs in the native
library (host front-end in C++, the search in HIP kernels for gfx950).
PyTorch supplies device memory (through the library's allocator hook) and
the HIP stream.  There is no CPU fallback: without ``libmpld.so`` importing
the binding raises, and without a gfx950 device the context call fails.
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from dataclasses import dataclass

import numpy as np

from . import _ffi
from ._ffi import (MPLD_BUDGET_EXHAUSTED, MPLD_FEASIBLE, MPLD_FORCE_DEVICE,  # noqa: F401
                   MPLD_FORCE_GLOBAL, MPLD_FORCE_LDS, MPLD_FORCE_WAVE, MPLD_INFEASIBLE,
                   MPLD_MARK_CONFLICTS, MPLD_MINIMIZE, MPLD_PLAIN, MPLD_SIMPLIFY, MPLD_SPLIT_HEAVY,
                   MPLD_STITCH_ORDER, MPLD_TRACE_HASH)

_lib = _ffi.load()

RECORD_DTYPE = np.dtype([("size", np.int32), ("status", np.int32), ("nodes", np.int64),
                         ("trace_hash", np.uint64), ("depth_at_stop", np.int32),
                         ("stitches", np.int32), ("first_node", np.int32),
                         ("num_edges", np.int32), ("conflicts", np.int32),
                         ("min_nodes", np.int32)])
assert RECORD_DTYPE.itemsize == ctypes.sizeof(_ffi.mpld_comp_record)


class MpldError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.mpld_error_string(code).decode()
        detail = (_lib.mpld_last_error() or b"").decode()
        super().__init__(f"{where}: {msg} ({code}): {detail}")


def _check(code: int, where: str) -> None:
    if code != 0:
        raise MpldError(code, where)


def mpld_abi_version() -> int:
    return int(_lib.mpld_abi_version())


def options(k: int, budget: int, flags: int = MPLD_SIMPLIFY,
            min_budget: int = 0) -> _ffi.mpld_options:
    return _ffi.mpld_options(ctypes.sizeof(_ffi.mpld_options), k, budget, flags, min_budget)


# ---- graphs -------------------------------------------------------------

@dataclass
class Graph:
    """A layout graph (nodes, conflict pairs, stitch pairs) in numpy arrays."""
    num_nodes: int
    ce: np.ndarray
    se: np.ndarray

    def view(self) -> _ffi.mpld_graph:
        self.ce = np.ascontiguousarray(self.ce, dtype=np.int32).reshape(-1, 2)
        self.se = np.ascontiguousarray(self.se, dtype=np.int32).reshape(-1, 2)
        return _ffi.mpld_graph(self.num_nodes, 0, len(self.ce), self.ce.ctypes.data,
                               len(self.se), self.se.ctypes.data)


def mpld_build_graph(rects: np.ndarray, dmin_nm: int, split_len_nm: int = 0) -> Graph:
    """Layout graph of rectangles (x0, y0, x1, y1) - see include/mpld.h."""
    r = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    h = ctypes.c_void_p()
    _check(_lib.mpld_build_graph(r.ctypes.data, len(r), dmin_nm, split_len_nm,
                                 ctypes.byref(h)), "mpld_build_graph")
    return _owned_graph(h)


def mpld_build_graph_device(ctx: "Context", rects: np.ndarray, dmin_nm: int,
                            split_len_nm: int = 0) -> Graph:
    """The same layout graph built on the context's device."""
    r = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    h = ctypes.c_void_p()
    _check(_lib.mpld_build_graph_device(ctx.handle, r.ctypes.data, len(r), dmin_nm,
                                        split_len_nm, ctypes.byref(h)),
           "mpld_build_graph_device")
    return _owned_graph(h)


def mpld_split_graph_device(ctx: "Context", g: Graph, k: int, simplify: bool = True):
    """Simplification and sub-graph split on the context's device.  Returns
    (removal_order, comp_of, [per-component global ids in local BFS order])."""
    n = g.num_nodes
    rem = np.zeros(max(n, 1), np.int32)
    comp_of = np.zeros(max(n, 1), np.int32)
    bfs = np.zeros(max(n, 1), np.int32)
    ptr = np.zeros(n + 1, np.int32)
    nrem, nc = ctypes.c_int32(), ctypes.c_int32()
    v = g.view()
    _check(_lib.mpld_split_graph_device(ctx.handle, ctypes.byref(v), k,
                                        MPLD_SIMPLIFY if simplify else 0, rem.ctypes.data,
                                        ctypes.byref(nrem), comp_of.ctypes.data, bfs.ctypes.data,
                                        ptr.ctypes.data, ctypes.byref(nc)),
           "mpld_split_graph_device")
    comps = [bfs[ptr[c]:ptr[c + 1]].copy() for c in range(nc.value)]
    return rem[: nrem.value].copy(), comp_of[:n].copy(), comps


def _owned_graph(h) -> Graph:
    try:
        v = _ffi.mpld_graph()
        _check(_lib.mpld_owned_graph_view(h, ctypes.byref(v)), "mpld_owned_graph_view")
        ce = np.ctypeslib.as_array((ctypes.c_int32 * (2 * v.num_ce)).from_address(v.ce)).copy() \
            if v.num_ce else np.zeros(0, np.int32)
        se = np.ctypeslib.as_array((ctypes.c_int32 * (2 * v.num_se)).from_address(v.se)).copy() \
            if v.num_se else np.zeros(0, np.int32)
        return Graph(v.num_nodes, ce.reshape(-1, 2), se.reshape(-1, 2))
    finally:
        _lib.mpld_owned_graph_free(h)


# ---- lifetimes ----------------------------------------------------------
# Servers, batches and contexts still open when the interpreter exits are
# closed by an exit hook, in that order (a server uses its context; a
# batch's and a context's device memory goes back through the torch
# allocator callback), while torch is still alive.  A destructor that runs
# during interpreter finalisation does nothing: calling the library then
# could call back into a torn-down torch.

_LIVE: dict = {0: weakref.WeakSet(), 1: weakref.WeakSet(), 2: weakref.WeakSet()}
_RANK = {"Server": 0, "Batch": 1, "Context": 2}


def _register(obj) -> None:
    _LIVE[_RANK[type(obj).__name__]].add(obj)
    ctx = getattr(obj, "ctx", None)
    if ctx is not None:   # a server or batch: its context closes it first
        children = getattr(ctx, "_children", None)
        if children is None:
            children = ctx._children = weakref.WeakSet()
        children.add(obj)


def _close_all() -> None:
    for rank in (0, 1, 2):
        for obj in list(_LIVE[rank]):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(_close_all)


def _finalizing() -> bool:
    return sys.is_finalizing()


# ---- context ------------------------------------------------------------

class _TorchAllocator:
    """Device memory from torch's caching allocator, kept alive by handle."""

    def __init__(self, device):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}

        def alloc(nbytes, _user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            p = t.data_ptr()
            self.live[p] = t
            return p

        def free(ptr, _user):
            self.live.pop(ptr, None)

        self._a = _ffi.ALLOC_FN(alloc)
        self._f = _ffi.FREE_FN(free)
        self.struct = _ffi.mpld_allocator(self._a, self._f, None)


class Context:
    """One device and one stream.  With use_torch the device memory comes
    from torch's caching allocator and the work runs on ``self.stream``, a
    torch stream of default priority (give it to torch.cuda.Event.record to
    time the library's launches)."""

    def __init__(self, device: int = 0, use_torch: bool = True):
        self.handle = ctypes.c_void_p()
        self._alloc = None
        self.stream = None
        handle = None
        alloc_ptr = None
        if use_torch:
            import torch
            dev = torch.device("cuda", device)
            self._alloc = _TorchAllocator(dev)
            alloc_ptr = ctypes.byref(self._alloc.struct)
            self.stream = torch.cuda.Stream(dev)
            handle = ctypes.c_void_p(self.stream.cuda_stream)
        _check(_lib.mpld_context_create(device, alloc_ptr, handle, ctypes.byref(self.handle)),
               "mpld_context_create")
        _register(self)

    def close(self):
        # servers and batches made on this context go first: they use its
        # stream and memory until they are destroyed
        for rank in (0, 1):
            for child in [c for c in list(getattr(self, "_children", ())) if _RANK[type(c).__name__] == rank]:
                try:
                    child.close()
                except Exception:
                    pass
        if self.handle:
            _lib.mpld_context_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        # at exit the module's globals may already be cleared (a lookup then
        # fails): the exit hook has closed every open object by then
        try:
            if self.handle and not _finalizing():
                self.close()
        except Exception:
            pass


def mpld_context_create(device: int = 0, use_torch: bool = True) -> Context:
    return Context(device, use_torch)


def mpld_context_destroy(ctx: Context) -> None:
    ctx.close()


# ---- results ------------------------------------------------------------

@dataclass
class Result:
    colors: np.ndarray        # int8 per node, -1 = uncolored
    component_of: np.ndarray  # int32 per node, -1 = removed by simplification
    components: np.ndarray    # RECORD_DTYPE per component
    stitches: int
    conflicts: int
    uncolored: int
    queue_us: float = 0.0     # serving: submit -> admission on the device
    total_us: float = 0.0     # serving: submit -> finished result


def _take_result(h) -> Result:
    try:
        n = ctypes.c_int32()
        pc = _lib.mpld_result_colors(h, ctypes.byref(n))
        colors = (np.ctypeslib.as_array((ctypes.c_int8 * n.value).from_address(pc)).copy()
                  if n.value else np.zeros(0, np.int8))
        po = _lib.mpld_result_component_of(h)
        comp_of = (np.ctypeslib.as_array((ctypes.c_int32 * n.value).from_address(po)).copy()
                   if n.value else np.zeros(0, np.int32))
        nc = _lib.mpld_result_num_components(h)
        if nc:
            pr = _lib.mpld_result_components(h)
            raw = (ctypes.c_uint8 * (nc * RECORD_DTYPE.itemsize)).from_address(pr)
            comps = np.frombuffer(bytes(raw), dtype=RECORD_DTYPE).copy()
        else:
            comps = np.zeros(0, RECORD_DTYPE)
        st, cn, un = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.mpld_result_totals(h, ctypes.byref(st), ctypes.byref(cn), ctypes.byref(un))
        q, t = ctypes.c_double(), ctypes.c_double()
        _lib.mpld_result_timing(h, ctypes.byref(q), ctypes.byref(t))
        return Result(colors, comp_of, comps, st.value, cn.value, un.value, q.value, t.value)
    finally:
        _lib.mpld_result_free(h)


def mpld_decompose(ctx: Context, g: Graph, k: int, budget: int,
                   flags: int = MPLD_SIMPLIFY, min_budget: int = 0) -> Result:
    opt = options(k, budget, flags, min_budget)
    view = g.view()
    h = ctypes.c_void_p()
    _check(_lib.mpld_decompose(ctx.handle, ctypes.byref(view), ctypes.byref(opt),
                               ctypes.byref(h)), "mpld_decompose")
    return _take_result(h)


class Batch:
    """Front-end + packed image resident on the device; solve repeatedly."""

    def __init__(self, ctx: Context, g: Graph, k: int, budget: int, flags: int = MPLD_SIMPLIFY,
                 min_budget: int = 0):
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        opt = options(k, budget, flags, min_budget)
        view = g.view()
        _check(_lib.mpld_batch_create(ctx.handle, ctypes.byref(view), ctypes.byref(opt),
                                      ctypes.byref(self.handle)), "mpld_batch_create")
        _register(self)

    def solve(self, plain: bool = False, direct: bool = False, split: bool = False,
              timed: bool = True, roundtrip: bool = False) -> None:
        flags = ((MPLD_PLAIN if plain else 0) | (_ffi.MPLD_DIRECT if direct else 0)
                 | (MPLD_SPLIT_HEAVY if split else 0) | (0 if timed else _ffi.MPLD_UNTIMED)
                 | (_ffi.MPLD_ROUNDTRIP if roundtrip else 0))
        _check(_lib.mpld_batch_solve(self.handle, flags), "mpld_batch_solve")

    def result(self) -> Result:
        h = ctypes.c_void_p()
        _check(_lib.mpld_batch_result(self.handle, ctypes.byref(h)), "mpld_batch_result")
        return _take_result(h)

    def info(self) -> dict:
        i = _ffi.mpld_batch_info()
        _check(_lib.mpld_batch_get_info(self.handle, ctypes.byref(i)), "mpld_batch_get_info")
        return {name: getattr(i, name) for name, _ in i._fields_}

    def autotune(self, reps: int = 5, cache_path: str | None = None) -> dict:
        t = _ffi.mpld_tune(ctypes.sizeof(_ffi.mpld_tune))
        _check(_lib.mpld_batch_autotune(self.handle, reps,
                                        cache_path.encode() if cache_path else None,
                                        ctypes.byref(t)), "mpld_batch_autotune")
        return {name: getattr(t, name) for name, _ in t._fields_ if name != "struct_size"}

    def get_tune(self) -> dict:
        t = _ffi.mpld_tune(ctypes.sizeof(_ffi.mpld_tune))
        _check(_lib.mpld_batch_get_tune(self.handle, ctypes.byref(t)), "mpld_batch_get_tune")
        return {name: getattr(t, name) for name, _ in t._fields_ if name != "struct_size"}

    def set_tune(self, **kw) -> None:
        t = _ffi.mpld_tune(ctypes.sizeof(_ffi.mpld_tune))
        _check(_lib.mpld_batch_get_tune(self.handle, ctypes.byref(t)), "mpld_batch_get_tune")
        for name, val in kw.items():
            setattr(t, name, val)
        _check(_lib.mpld_batch_set_tune(self.handle, ctypes.byref(t)), "mpld_batch_set_tune")

    def close(self):
        if self.handle:
            _lib.mpld_batch_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        # at exit the module's globals may already be cleared (a lookup then
        # fails): the exit hook has closed every open object by then
        try:
            if self.handle and not _finalizing():
                self.close()
        except Exception:
            pass


def mpld_batch_create(ctx: Context, g: Graph, k: int, budget: int,
                      flags: int = MPLD_SIMPLIFY) -> Batch:
    return Batch(ctx, g, k, budget, flags)


def mpld_batch_solve(b: Batch, plain: bool = False, direct: bool = False,
                     split: bool = False, timed: bool = True) -> None:
    b.solve(plain, direct, split, timed)


def mpld_batch_result(b: Batch) -> Result:
    return b.result()


def mpld_batch_get_info(b: Batch) -> dict:
    return b.info()


def mpld_batch_free(b: Batch) -> None:
    b.close()


def mpld_batch_autotune(b: Batch, reps: int = 5, cache_path: str | None = None) -> dict:
    return b.autotune(reps, cache_path)


def mpld_batch_get_tune(b: Batch) -> dict:
    return b.get_tune()


def mpld_batch_set_tune(b: Batch, **kw) -> None:
    b.set_tune(**kw)


def _solve_components(fn, name, ctx: Context, comps, k: int, budget: int, flags: int,
                      min_budget: int):
    arrs = []
    cs = (_ffi.mpld_component * max(len(comps), 1))()
    total = 0
    for i, (n, e) in enumerate(comps):
        a = np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))
        arrs.append(a)
        cs[i] = _ffi.mpld_component(n, 0, len(a), a.ctypes.data)
        total += n
    recs = (_ffi.mpld_comp_record * max(len(comps), 1))()
    colors = np.zeros(max(total, 1), dtype=np.int8)
    opt = options(k, budget, flags, min_budget)
    _check(fn(ctx.handle, cs, len(comps), ctypes.byref(opt), recs, colors.ctypes.data), name)
    out = np.frombuffer(bytes(recs), dtype=RECORD_DTYPE)[: len(comps)].copy()
    per, off = [], 0
    for n, _ in comps:
        per.append(colors[off: off + n].copy())
        off += n
    return out, per


def mpld_solve_components(ctx: Context, comps, k: int, budget: int, flags: int = 0,
                          min_budget: int = 0):
    """comps: list of (n, edges [m, 2]) in local numbering.  Returns
    (records RECORD_DTYPE[count], list of per-component int8 colors)."""
    return _solve_components(_lib.mpld_solve_components, "mpld_solve_components", ctx, comps, k,
                             budget, flags, min_budget)


def mpld_solve_components_noalloc(ctx: Context, comps, k: int, budget: int, flags: int = 0):
    """As mpld_solve_components, through the entry point that allocates
    nothing (components of at most 64 nodes, fixed device scratch)."""
    return _solve_components(_lib.mpld_solve_components_noalloc, "mpld_solve_components_noalloc",
                             ctx, comps, k, budget, flags, 0)


def mpld_measure_lds_read_rate(ctx: Context, bytes_per_lane: int = 16, iters: int = 2000) -> dict:
    """The chip's LDS read rate (ds_read_b64 / ds_read_b128 on every CU)."""
    gbps = ctypes.c_double()
    per = ctypes.c_double()
    _check(_lib.mpld_measure_lds_read_rate(ctx.handle, bytes_per_lane, iters, ctypes.byref(gbps),
                                           ctypes.byref(per)), "mpld_measure_lds_read_rate")
    return {"GBps": gbps.value, "bytes_per_clock_per_cu": per.value}


def mpld_measure_launch_floor(ctx: Context, grid: int, block: int = 256, reps: int = 200) -> float:
    """Microseconds per launch of an empty kernel of `grid` x `block`
    lanes, launched back to back on the context stream."""
    us = ctypes.c_double()
    _check(_lib.mpld_measure_launch_floor(ctx.handle, grid, block, reps, ctypes.byref(us)),
           "mpld_measure_launch_floor")
    return us.value


def mpld_measure_touch_floor(ctx: Context, grid: int, block: int = 256, reps: int = 200) -> float:
    """Microseconds per launch of a kernel of `grid` x `block` lanes whose
    every wave reads 64 bytes and writes 8, launched back to back."""
    us = ctypes.c_double()
    _check(_lib.mpld_measure_touch_floor(ctx.handle, grid, block, reps, ctypes.byref(us)),
           "mpld_measure_touch_floor")
    return us.value


# ---- serving ----------------------------------------------------------------

class Server:
    """Continuous-batching server on a context (see include/mpld.h)."""

    def __init__(self, ctx: Context, max_components: int = 0, arena_bytes: int = 0,
                 slice_nodes: int = 0, host_threads: int = 0, graph_builders: int = 0,
                 device_split: bool = True):
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        o = _ffi.mpld_server_options(ctypes.sizeof(_ffi.mpld_server_options), max_components,
                                     arena_bytes, slice_nodes, host_threads, graph_builders,
                                     0 if device_split else -1, 0)
        _check(_lib.mpld_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(self.handle)),
               "mpld_server_create")
        _register(self)

    def submit_layout(self, rects: np.ndarray, dmin_nm: int, split_len_nm: int, k: int,
                      budget: int, flags: int = MPLD_SIMPLIFY, min_budget: int = 0) -> int:
        r = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
        opt = options(k, budget, flags, min_budget)
        t = ctypes.c_uint64()
        _check(_lib.mpld_server_submit_layout(self.handle, r.ctypes.data, len(r), dmin_nm,
                                              split_len_nm, ctypes.byref(opt), ctypes.byref(t)),
               "mpld_server_submit_layout")
        return t.value

    def submit(self, g: Graph, k: int, budget: int, flags: int = MPLD_SIMPLIFY,
               min_budget: int = 0) -> int:
        opt = options(k, budget, flags, min_budget)
        view = g.view()
        t = ctypes.c_uint64()
        _check(_lib.mpld_server_submit(self.handle, ctypes.byref(view), ctypes.byref(opt),
                                       ctypes.byref(t)), "mpld_server_submit")
        return t.value

    def poll(self, ticket: int):
        h = ctypes.c_void_p()
        rc = _lib.mpld_server_poll(self.handle, ticket, ctypes.byref(h))
        if rc == _ffi.MPLD_E_NOT_READY:
            return None
        _check(rc, "mpld_server_poll")
        return _take_result(h)

    def wait(self, ticket: int, timeout_us: int = -1):
        h = ctypes.c_void_p()
        rc = _lib.mpld_server_wait(self.handle, ticket, timeout_us, ctypes.byref(h))
        if rc == _ffi.MPLD_E_NOT_READY:
            return None
        _check(rc, "mpld_server_wait")
        return _take_result(h)

    def stats(self) -> dict:
        st = _ffi.mpld_server_stats()
        _check(_lib.mpld_server_get_stats(self.handle, ctypes.byref(st)), "mpld_server_get_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if self.handle:
            _lib.mpld_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        # at exit the module's globals may already be cleared (a lookup then
        # fails): the exit hook has closed every open object by then
        try:
            if self.handle and not _finalizing():
                self.close()
        except Exception:
            pass


def mpld_server_create(ctx: Context, **kw) -> Server:
    return Server(ctx, **kw)


def mpld_server_submit_layout(s: Server, rects, dmin_nm: int, split_len_nm: int, k: int,
                              budget: int, flags: int = MPLD_SIMPLIFY) -> int:
    return s.submit_layout(rects, dmin_nm, split_len_nm, k, budget, flags)


def mpld_server_submit(s: Server, g: Graph, k: int, budget: int, flags: int = MPLD_SIMPLIFY) -> int:
    return s.submit(g, k, budget, flags)


def mpld_server_poll(s: Server, ticket: int):
    return s.poll(ticket)


def mpld_server_wait(s: Server, ticket: int, timeout_us: int = -1):
    return s.wait(ticket, timeout_us)


def mpld_server_get_stats(s: Server) -> dict:
    return s.stats()


def mpld_server_destroy(s: Server) -> None:
    s.close()
