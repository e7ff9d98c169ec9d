"""Seeded synthetic inputs: rectangle layouts and serving request traces.

This package only produces inputs (see ``layoutgen.h`` for the exact
definition of every draw).  It contains none of the decomposition method's
arithmetic and is shared by the product library's callers (bench, tests) and
by the oracle's tests.  The paper's ISCAS layouts (Sec. 3, Table 1) are not
available; these generators stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblayoutgen.so")
_lib = None


class LgParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("side", ctypes.c_int32),
                ("width", ctypes.c_int32), ("len_min", ctypes.c_int32),
                ("len_max", ctypes.c_int32), ("max_attempts", ctypes.c_int32)]


def build() -> str:
    """Compile liblayoutgen.so in place (plain C, host only)."""
    src = os.path.join(_HERE, "layoutgen.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
                           "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; call workload.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.lg_u64.restype = ctypes.c_uint64
        lib.lg_u64.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.lg_generate.restype = ctypes.c_int32
        lib.lg_generate.argtypes = [ctypes.POINTER(LgParams), ctypes.c_uint64,
                                    ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
        lib.lg_request_trace.restype = ctypes.c_int32
        lib.lg_request_trace.argtypes = [
            ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def splitmix64(seed: int, count: int) -> list[int]:
    """`count` consecutive SplitMix64 outputs from state `seed`."""
    lib = _load()
    st = ctypes.c_uint64(seed)
    return [lib.lg_u64(ctypes.byref(st)) for _ in range(count)]


def generate(n: int, side: int, seed: int, width: int = 20, len_min: int = 40,
             len_max: int = 200, max_attempts: int = 1000):
    """Returns (rects int32 [placed, 4] as x0,y0,x1,y1; skipped count)."""
    lib = _load()
    p = LgParams(n, side, width, len_min, len_max, max_attempts)
    out = np.zeros((max(n, 1), 4), dtype=np.int32)
    placed = ctypes.c_int32(0)
    skipped = ctypes.c_int32(0)
    rc = lib.lg_generate(ctypes.byref(p), ctypes.c_uint64(seed),
                         out.ctypes.data, ctypes.byref(placed),
                         ctypes.byref(skipped))
    if rc != 0:
        raise ValueError(f"lg_generate failed with {rc}")
    return np.ascontiguousarray(out[: placed.value]), skipped.value


def request_trace(seed: int, count: int, rate: float = 500.0, n_min: int = 100,
                  n_max: int = 50000, base_side: int = 3000, base_n: int = 300):
    """Returns dict of numpy arrays: arrival_s, n_rects, side_nm, seed."""
    lib = _load()
    arr = np.zeros(count, dtype=np.float64)
    nr = np.zeros(count, dtype=np.int32)
    sd = np.zeros(count, dtype=np.int32)
    ls = np.zeros(count, dtype=np.uint64)
    rc = lib.lg_request_trace(ctypes.c_uint64(seed), count, rate, n_min, n_max,
                              base_side, base_n, arr.ctypes.data,
                              nr.ctypes.data, sd.ctypes.data, ls.ctypes.data)
    if rc != 0:
        raise ValueError(f"lg_request_trace failed with {rc}")
    return {"arrival_s": arr, "n_rects": nr, "side_nm": sd, "seed": ls}


def random_component(n: int, avg_degree: float, seed: int) -> np.ndarray:
    """Connected random graph for latency probes: the path 0-1-...-(n-1) plus
    uniformly random extra pairs (numpy PCG64, `seed`) until n*avg_degree/2
    distinct pairs.  Returns int32 [m, 2] pairs (u < v), sorted."""
    rng = np.random.default_rng(seed)
    m = int(n * avg_degree / 2)
    e = set((i, i + 1) for i in range(n - 1))
    while len(e) < m:
        a, b = rng.integers(0, n, 2)
        if a != b:
            e.add((int(min(a, b)), int(max(a, b))))
    return np.array(sorted(e), dtype=np.int32).reshape(-1, 2)
