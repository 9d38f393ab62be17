"""ORACLE (test infrastructure only): ctypes binding of ``rrg_oracle.c``, the serial
statement of the exploration support (Philox sampling, obstacle tests, radius
neighbours with exact segment tests, FP32 costs and heuristic).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rrg_oracle.c")
_LIB = os.path.join(_HERE, "librrg_oracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fPIC", "-shared",
          "-std=c11"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc"] + CFLAGS + [_SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    cint, dbl = ctypes.c_int, ctypes.c_double
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
    lib.orc_candidate.restype = None
    lib.orc_candidate.argtypes = [cint, u64, u32, u64, vp]
    lib.orc_point_blocked.restype = cint
    lib.orc_point_blocked.argtypes = [cint, vp, cint, vp, vp, vp]
    lib.orc_segment_blocked.restype = cint
    lib.orc_segment_blocked.argtypes = [cint, vp, vp, cint, vp, vp, vp]
    lib.orc_sample.restype = cint
    lib.orc_sample.argtypes = [cint, u64, u32, ctypes.POINTER(u64), i64, cint, vp, vp, vp, i64, vp]
    lib.orc_build_rows.restype = i64
    lib.orc_build_rows.argtypes = [cint, i64, i64, vp, dbl, cint, vp, vp, vp, vp, vp, vp, i64]
    lib.orc_heuristic.restype = None
    lib.orc_heuristic.argtypes = [cint, i64, vp, vp, vp]
    _lib = lib
    return lib


def _obs_arrays(obs, d):
    if obs is None or len(obs.kind) == 0:
        z = np.zeros(1, np.int32)
        return 0, z, np.zeros(d), np.zeros(d)
    kind = np.ascontiguousarray(obs.kind, np.int32)
    centre = np.ascontiguousarray(obs.centre, np.float64)
    size = np.ascontiguousarray(obs.size, np.float64)
    return len(kind), kind, centre, size


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    load().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def candidate(d: int, seed: int, stream: int, k: int) -> np.ndarray:
    x = np.zeros(d, np.float64)
    load().orc_candidate(d, seed, stream, k, x.ctypes.data)
    return x


def point_blocked(x, obs) -> bool:
    x = np.ascontiguousarray(x, np.float64)
    m, kind, centre, size = _obs_arrays(obs, len(x))
    return bool(load().orc_point_blocked(len(x), x.ctypes.data, m, kind.ctypes.data, centre.ctypes.data,
                                         size.ctypes.data))


def segment_blocked(a, b, obs) -> bool:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    m, kind, centre, size = _obs_arrays(obs, len(a))
    return bool(load().orc_segment_blocked(len(a), a.ctypes.data, b.ctypes.data, m, kind.ctypes.data,
                                           centre.ctypes.data, size.ctypes.data))


def sample(d: int, seed: int, stream: int, counter: int, count: int, obs,
           max_candidates: int = 1 << 40) -> Tuple[np.ndarray, int]:
    """`count` free samples from candidate `counter` on; returns (points, next counter)."""
    pts = np.zeros((max(count, 1), d), np.float64)
    m, kind, centre, size = _obs_arrays(obs, d)
    c = ctypes.c_uint64(counter)
    rc = load().orc_sample(d, seed, stream, ctypes.byref(c), count, m, kind.ctypes.data, centre.ctypes.data,
                           size.ctypes.data, max_candidates, pts.ctypes.data)
    if rc != 0:
        raise RuntimeError("orc_sample failed")
    return pts[:count], int(c.value)


def build_rows(pts: np.ndarray, n_old: int, r: float, obs):
    """Forward rows (row_ptr, col, cost) of vertices n_old .. len(pts)-1."""
    pts = np.ascontiguousarray(pts, np.float64)
    n, d = pts.shape
    m, kind, centre, size = _obs_arrays(obs, d)
    cap = max(1024, (n - n_old) * 64)
    while True:
        row_ptr = np.zeros(n - n_old + 1, np.int64)
        col = np.zeros(cap, np.int32)
        cost = np.zeros(cap, np.float32)
        got = load().orc_build_rows(d, n_old, n, pts.ctypes.data, r, m, kind.ctypes.data, centre.ctypes.data,
                                    size.ctypes.data, row_ptr.ctypes.data, col.ctypes.data, cost.ctypes.data, cap)
        if got >= 0:
            return row_ptr, col[:got].copy(), cost[:got].copy()
        cap *= 4


def heuristic(pts: np.ndarray, goal) -> np.ndarray:
    pts = np.ascontiguousarray(pts, np.float64)
    goal = np.ascontiguousarray(goal, np.float64)
    n, d = pts.shape
    h = np.zeros(max(n, 1), np.float32)
    load().orc_heuristic(d, n, pts.ctypes.data, goal.ctypes.data, h.ctypes.data)
    return h[:n]
