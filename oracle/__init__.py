"""ORACLE (test infrastructure only): ctypes binding of the serial CPU statement of
PI-RRT#'s exploitation phase in ``pirrt_oracle.c``.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It shares no code with the GPU library and never stands in for it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pirrt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, ENOTCONVERGED = 0, -1, -2, -4

# Flags for a binary32 statement with no contraction, no fast-math reassociation
# and SSE arithmetic (no x87 excess precision).
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fPIC",
          "-shared", "-std=c11"]


def build(force: bool = False, defines=(), out: Optional[str] = None) -> str:
    """Compiles the oracle with gcc.  `defines` adds -D flags (used by the tests
    that plant mistakes in a separate copy of the oracle)."""
    out = out or _LIB
    if force or defines or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc"] + CFLAGS + ["-D%s" % d for d in defines] + [_SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("edges_examined", ctypes.c_int64),
                ("sum_P", ctypes.c_int64), ("sum_D", ctypes.c_int64),
                ("changed_total", ctypes.c_int64), ("mark_edges", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def load(path: Optional[str] = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB
    if path is None and (not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(p)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = []
    lib.orc_destroy.restype = None
    lib.orc_destroy.argtypes = [vp]
    lib.orc_num_vertices.restype = i64
    lib.orc_num_vertices.argtypes = [vp]
    lib.orc_num_edges.restype = i64
    lib.orc_num_edges.argtypes = [vp]
    lib.orc_insert.restype = ctypes.c_int
    lib.orc_insert.argtypes = [vp, i32, vp, vp, vp]
    lib.orc_set_state.restype = ctypes.c_int
    lib.orc_set_state.argtypes = [vp, vp, vp, vp]
    lib.orc_get_state.restype = None
    lib.orc_get_state.argtypes = [vp, vp, vp, vp]
    lib.orc_get_adjacency.restype = None
    lib.orc_get_adjacency.argtypes = [vp, vp, vp, vp]
    lib.orc_replan.restype = ctypes.c_int
    lib.orc_replan.argtypes = [vp, i32, i32, vp, ctypes.c_int, i32, ctypes.POINTER(Stats)]
    lib.orc_replan_mode.restype = ctypes.c_int
    lib.orc_replan_mode.argtypes = [vp, i32, i32, vp, ctypes.c_int, ctypes.c_int, i32, ctypes.POINTER(Stats)]
    lib.orc_evaluate.restype = i64
    lib.orc_evaluate.argtypes = [vp, i32]
    if path is None:
        _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


@dataclass
class State:
    g: np.ndarray
    parent: np.ndarray
    pcost: np.ndarray


class Graph:
    """The oracle's graph and policy: plain adjacency lists plus SoA g/parent/pcost."""

    def __init__(self, lib=None):
        self._lib = lib or load()
        self._h = self._lib.orc_create()
        if not self._h:
            raise MemoryError("orc_create")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def n(self) -> int:
        return int(self._lib.orc_num_vertices(self._h))

    @property
    def nnz(self) -> int:
        return int(self._lib.orc_num_edges(self._h))

    def insert(self, row_ptr, col, cost) -> int:
        row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        cost = np.ascontiguousarray(cost, np.float32)
        n_new = len(row_ptr) - 1
        return int(self._lib.orc_insert(self._h, n_new, row_ptr.ctypes.data,
                                        _ptr(col) if len(col) else None,
                                        _ptr(cost) if len(cost) else None))

    def insert_batch(self, batch) -> int:
        return self.insert(batch.row_ptr, batch.col, batch.cost)

    def state(self) -> State:
        n = self.n
        g = np.empty(n, np.float32)
        p = np.empty(n, np.int32)
        c = np.empty(n, np.float32)
        self._lib.orc_get_state(self._h, _ptr(g), _ptr(p), _ptr(c))
        return State(g, p, c)

    def set_state(self, g, parent, pcost) -> int:
        g = np.ascontiguousarray(g, np.float32)
        parent = np.ascontiguousarray(parent, np.int32)
        pcost = np.ascontiguousarray(pcost, np.float32)
        return int(self._lib.orc_set_state(self._h, _ptr(g), _ptr(parent), _ptr(pcost)))

    def adjacency(self):
        """(ptr int64[n+1], nbr int32[nnz], cost float32[nnz]) of the undirected graph."""
        n = self.n
        ptr = np.empty(n + 1, np.int64)
        nbr = np.empty(max(self.nnz, 1), np.int32)
        cst = np.empty(max(self.nnz, 1), np.float32)
        self._lib.orc_get_adjacency(self._h, _ptr(ptr), _ptr(nbr), _ptr(cst))
        return ptr, nbr[: self.nnz], cst[: self.nnz]

    def replan(self, root: int, goal: int, h=None, prune: bool = True, max_iters: int = 0,
               lookahead: bool = False, truncated: bool = False):
        """Returns (rc, stats dict).  The policy is updated in place.  lookahead selects
        the narrowed Improve domain, truncated the truncated Evaluate (see
        orc_replan_mode); both together are rejected."""
        st = Stats()
        hh = None if h is None else np.ascontiguousarray(h, np.float32)
        mode = (1 if lookahead else 0) | (2 if truncated else 0)
        rc = self._lib.orc_replan_mode(self._h, int(root), int(goal), _ptr(hh), int(bool(prune)),
                                       mode, int(max_iters), ctypes.byref(st))
        return int(rc), st.as_dict()

    def evaluate(self, root: int) -> int:
        return int(self._lib.orc_evaluate(self._h, int(root)))
