"""ctypes binding of libpirrt.so, the gfx950 Replan library declared in include/pirrt.h.

The functions keep the C names (``pirrt_graph_create``, ``pirrt_insert_batch``,
``pirrt_replan`` ...) and only marshal arguments: numpy arrays are passed as host
buffers, torch tensors on a ROCm device as device buffers (their ``data_ptr``).
Every step of the computation runs in the library's HIP kernels; when the library
is not built, loading fails loudly instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpirrt.so")

PIRRT_OK, PIRRT_EINVAL, PIRRT_ENOMEM, PIRRT_EDEVICE, PIRRT_ENOTCONVERGED = 0, -1, -2, -3, -4
PIRRT_MEM_HOST, PIRRT_MEM_DEVICE = 0, 1
PIRRT_NO_PRUNE, PIRRT_TIMING, PIRRT_LOOKAHEAD, PIRRT_TRUNCATED = 1, 2, 4, 8
PIRRT_MLP_NOALLOC_MAX_BATCH = 8192

EXPORTS = [
    "pirrt_config_init", "pirrt_graph_create", "pirrt_graph_destroy", "pirrt_insert_batch", "pirrt_replan",
    "pirrt_get_policy", "pirrt_set_policy", "pirrt_snapshot_save", "pirrt_snapshot_restore",
    "pirrt_get_adjacency", "pirrt_num_vertices", "pirrt_num_edges", "pirrt_last_error", "pirrt_strerror",
    "pirrt_batch_create", "pirrt_batch_destroy", "pirrt_batch_add_problem", "pirrt_batch_num_problems",
    "pirrt_batch_num_vertices", "pirrt_batch_num_edges", "pirrt_batch_problem_offset", "pirrt_batch_replan",
    "pirrt_batch_get_policy", "pirrt_batch_snapshot_save", "pirrt_batch_snapshot_restore",
    "pirrt_batch_last_error",
    "pirrt_rrg_create", "pirrt_rrg_destroy", "pirrt_rrg_num_points", "pirrt_rrg_add_points", "pirrt_rrg_sample",
    "pirrt_rrg_get_points", "pirrt_rrg_rows", "pirrt_rrg_connect", "pirrt_rrg_connect_problem",
    "pirrt_rrg_heuristic", "pirrt_rrg_last_error",
    "pirrt_mlp_num_params", "pirrt_mlp_create", "pirrt_mlp_destroy", "pirrt_mlp_set_params", "pirrt_mlp_get_params",
    "pirrt_mlp_forward", "pirrt_mlp_gradients", "pirrt_mlp_train_step", "pirrt_mlp_last_error",
    "pirrt_mlp_in_dim", "pirrt_rrg_sample_learned", "pirrt_tune", "pirrt_batch_tune",
    "pirrt_mlp_forward_noalloc", "pirrt_batch_insert", "pirrt_state_size", "pirrt_state_save",
    "pirrt_state_restore", "pirrt_promising_count",
]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class pirrt_config(ctypes.Structure):
    _fields_ = [("vertex_capacity", ctypes.c_int64), ("edge_capacity", ctypes.c_int64),
                ("hip_stream", ctypes.c_void_p), ("max_iters", ctypes.c_int32), ("device", ctypes.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p)]


class TorchAllocator:
    """Allocator callbacks of pirrt_config that take device memory from torch's
    caching allocator on a given device and stream (marshalling only: the library
    calls them when its storage grows)."""

    def __init__(self, device: int, stream: Optional[int]):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device < 0 else device
        self.stream = stream or 0
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except RuntimeError:
            return None

    def _free(self, ptr, ctx):
        if ptr:
            self._torch.cuda.caching_allocator_delete(ptr)


class pirrt_rrg_config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n_obstacles", ctypes.c_int32), ("kind", ctypes.c_void_p),
                ("centre", ctypes.c_void_p), ("size", ctypes.c_void_p), ("point_capacity", ctypes.c_int64),
                ("hip_stream", ctypes.c_void_p), ("device", ctypes.c_int32)]


class pirrt_mlp_config(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("hip_stream", ctypes.c_void_p), ("device", ctypes.c_int32)]


class pirrt_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("on_host", ctypes.c_int32),
                ("edges_examined", ctypes.c_int64), ("sum_P", ctypes.c_int64), ("sum_D", ctypes.c_int64),
                ("changed_total", ctypes.c_int64), ("ms_total", ctypes.c_double),
                ("ms_evaluate", ctypes.c_double), ("ms_mark", ctypes.c_double), ("ms_improve", ctypes.c_double),
                ("improve_launches", ctypes.c_int32), ("mark_launches", ctypes.c_int32),
                ("evaluate_calls", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mark_edges", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class PirrtError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


_lib = None


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Loads libpirrt.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libpirrt.so is not built (%s); run __graft_entry__.build()" % p)
    lib = ctypes.CDLL(p)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    cint = ctypes.c_int
    sig = {
        "pirrt_config_init": (cint, [ctypes.POINTER(pirrt_config)]),
        "pirrt_graph_create": (cint, [ctypes.POINTER(vp), ctypes.POINTER(pirrt_config)]),
        "pirrt_graph_destroy": (cint, [vp]),
        "pirrt_insert_batch": (cint, [vp, i32, vp, vp, vp, cint]),
        "pirrt_replan": (cint, [vp, i32, i32, vp, u32, vp, vp, cint, ctypes.POINTER(pirrt_stats)]),
        "pirrt_get_policy": (cint, [vp, vp, vp, vp, cint]),
        "pirrt_set_policy": (cint, [vp, vp, vp, vp, cint]),
        "pirrt_snapshot_save": (cint, [vp]),
        "pirrt_snapshot_restore": (cint, [vp]),
        "pirrt_get_adjacency": (cint, [vp, vp, vp, vp, cint]),
        "pirrt_state_size": (i64, [vp]),
        "pirrt_promising_count": (cint, [vp, i32, vp, i64, i64, cint, ctypes.POINTER(i64)]),
        "pirrt_state_save": (cint, [vp, vp, i64]),
        "pirrt_state_restore": (cint, [vp, vp, i64]),
        "pirrt_num_vertices": (i64, [vp]),
        "pirrt_num_edges": (i64, [vp]),
        "pirrt_last_error": (ctypes.c_char_p, [vp]),
        "pirrt_strerror": (ctypes.c_char_p, [cint]),
        "pirrt_batch_create": (cint, [ctypes.POINTER(vp), ctypes.POINTER(pirrt_config)]),
        "pirrt_batch_destroy": (cint, [vp]),
        "pirrt_batch_add_problem": (cint, [vp, i32, vp, vp, vp, cint, ctypes.POINTER(i32)]),
        "pirrt_batch_insert": (cint, [vp, i32, vp, vp, vp, vp, vp, cint]),
        "pirrt_batch_num_problems": (i32, [vp]),
        "pirrt_batch_num_vertices": (i64, [vp]),
        "pirrt_batch_num_edges": (i64, [vp]),
        "pirrt_batch_problem_offset": (i64, [vp, i32]),
        "pirrt_batch_replan": (cint, [vp, vp, vp, vp, u32, vp, vp, cint, vp]),
        "pirrt_batch_get_policy": (cint, [vp, vp, vp, vp, cint]),
        "pirrt_batch_snapshot_save": (cint, [vp]),
        "pirrt_batch_snapshot_restore": (cint, [vp]),
        "pirrt_batch_last_error": (ctypes.c_char_p, [vp]),
        "pirrt_rrg_create": (cint, [ctypes.POINTER(vp), ctypes.POINTER(pirrt_rrg_config)]),
        "pirrt_rrg_destroy": (cint, [vp]),
        "pirrt_rrg_num_points": (i64, [vp]),
        "pirrt_rrg_add_points": (cint, [vp, i32, vp, cint]),
        "pirrt_rrg_sample": (cint, [vp, ctypes.c_uint64, u32, ctypes.POINTER(ctypes.c_uint64), i32]),
        "pirrt_rrg_get_points": (cint, [vp, i64, i64, vp, cint]),
        "pirrt_rrg_rows": (cint, [vp, i64, ctypes.c_double, vp, vp, vp, i64, ctypes.POINTER(i64), cint]),
        "pirrt_rrg_connect": (cint, [vp, i64, ctypes.c_double, vp]),
        "pirrt_rrg_connect_problem": (cint, [vp, ctypes.c_double, vp, ctypes.POINTER(i32)]),
        "pirrt_rrg_heuristic": (cint, [vp, i64, vp, cint]),
        "pirrt_rrg_last_error": (ctypes.c_char_p, [vp]),
        "pirrt_mlp_num_params": (i64, []),
        "pirrt_mlp_create": (cint, [ctypes.POINTER(vp), ctypes.POINTER(pirrt_mlp_config)]),
        "pirrt_mlp_destroy": (cint, [vp]),
        "pirrt_mlp_set_params": (cint, [vp, vp, cint]),
        "pirrt_mlp_get_params": (cint, [vp, vp, cint]),
        "pirrt_mlp_forward": (cint, [vp, i32, vp, vp, cint]),
        "pirrt_mlp_forward_noalloc": (cint, [vp, i32, vp, vp]),
        "pirrt_mlp_gradients": (cint, [vp, i32, vp, vp, vp, ctypes.POINTER(ctypes.c_float), cint]),
        "pirrt_mlp_train_step": (cint, [vp, i32, vp, vp, ctypes.POINTER(ctypes.c_float), cint]),
        "pirrt_mlp_last_error": (ctypes.c_char_p, [vp]),
        "pirrt_mlp_in_dim": (i32, [vp]),
        "pirrt_rrg_sample_learned": (cint, [vp, vp, vp, i32, ctypes.c_uint64, u32, ctypes.POINTER(ctypes.c_uint64),
                                            i32, i32]),
        "pirrt_tune": (cint, [vp, i32, i32, vp, u32, cint, ctypes.POINTER(i32)]),
        "pirrt_batch_tune": (cint, [vp, vp, vp, vp, u32, cint, ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _strerror(code: int) -> str:
    try:
        return load().pirrt_strerror(code).decode()
    except Exception:  # library missing: still format the error
        return "error"


def _is_device(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


def _mem_kind(*arrays) -> int:
    kinds = {_is_device(a) for a in arrays if a is not None}
    if len(kinds) > 1:
        raise ValueError("mix of host and device buffers in one call")
    return PIRRT_MEM_DEVICE if kinds == {True} else PIRRT_MEM_HOST


def _check_dtype(x, np_dtype, torch_name):
    if x is None:
        return x
    if hasattr(x, "data_ptr"):
        if str(x.dtype) != "torch." + torch_name or not x.is_contiguous():
            raise TypeError("expected a contiguous torch.%s tensor" % torch_name)
        return x
    return np.ascontiguousarray(x, dtype=np_dtype)


class Graph:
    """One pirrt_graph handle.  `stream` is a hipStream_t as an int (for example
    ``torch.cuda.current_stream().cuda_stream``) or None for the null stream."""

    def __init__(self, stream: Optional[int] = None, device: int = -1, max_iters: int = 0,
                 vertex_capacity: int = 0, edge_capacity: int = 0, lib: Optional[ctypes.CDLL] = None,
                 torch_allocator: bool = False):
        self._lib = lib or load()
        cfg = pirrt_config()
        self._lib.pirrt_config_init(ctypes.byref(cfg))
        cfg.vertex_capacity = vertex_capacity
        cfg.edge_capacity = edge_capacity
        cfg.hip_stream = stream or None
        cfg.max_iters = max_iters
        cfg.device = device
        self._alloc = TorchAllocator(device, stream) if torch_allocator else None
        if self._alloc is not None:
            cfg.alloc = self._alloc.alloc
            cfg.free = self._alloc.free
        h = ctypes.c_void_p()
        rc = self._lib.pirrt_graph_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_last_error(None).decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.pirrt_graph_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    def _check(self, rc: int, allow=()):
        if rc != PIRRT_OK and rc not in allow:
            raise PirrtError(rc, self._lib.pirrt_last_error(self._h).decode())
        return rc

    @property
    def n(self) -> int:
        return int(self._lib.pirrt_num_vertices(self._h))

    @property
    def nnz(self) -> int:
        return int(self._lib.pirrt_num_edges(self._h))

    def insert_batch(self, row_ptr, col, cost) -> int:
        row_ptr = _check_dtype(row_ptr, np.int64, "int64")
        col = _check_dtype(col, np.int32, "int32")
        cost = _check_dtype(cost, np.float32, "float32")
        kind = _mem_kind(row_ptr, col, cost)
        n_new = int(row_ptr.shape[0]) - 1
        rc = self._lib.pirrt_insert_batch(self._h, n_new, _ptr(row_ptr), _ptr(col) if len(col) else None,
                                          _ptr(cost) if len(cost) else None, kind)
        return self._check(rc)

    def insert_rows(self, batch) -> int:
        """Inserts a workload batch (row_ptr / col / cost arrays)."""
        return self.insert_batch(batch.row_ptr, batch.col, batch.cost)

    def replan(self, root: int, goal: int, h=None, prune: bool = True, timing: bool = False,
               g_out=None, parent_out=None, allow_not_converged: bool = False, lookahead: bool = False,
               truncated: bool = False):
        """Runs Replan.  Outputs are numpy arrays unless device buffers are given
        (torch tensors on the GPU) or h is a device tensor.  lookahead selects the
        narrowed Improve domain (PIRRT_LOOKAHEAD), truncated the truncated Evaluate
        (PIRRT_TRUNCATED)."""
        h = _check_dtype(h, np.float32, "float32")
        n = self.n
        if g_out is None and parent_out is None and _is_device(h):
            import torch
            g_out = torch.empty(n, dtype=torch.float32, device=h.device)
            parent_out = torch.empty(n, dtype=torch.int32, device=h.device)
        if g_out is None and parent_out is None:
            g_out = np.empty(n, np.float32)
            parent_out = np.empty(n, np.int32)
        kind = _mem_kind(h, g_out, parent_out)
        flags = ((0 if prune else PIRRT_NO_PRUNE) | (PIRRT_TIMING if timing else 0) |
                 (PIRRT_LOOKAHEAD if lookahead else 0) | (PIRRT_TRUNCATED if truncated else 0))
        st = pirrt_stats()
        rc = self._lib.pirrt_replan(self._h, int(root), int(goal), _ptr(h), flags, _ptr(g_out), _ptr(parent_out),
                                    kind, ctypes.byref(st))
        self._check(rc, allow=(PIRRT_ENOTCONVERGED,) if allow_not_converged else ())
        d = st.as_dict()
        d["rc"] = rc
        return g_out, parent_out, d

    def tune(self, root: int, goal: int, h=None, prune: bool = True, lookahead: bool = False,
             truncated: bool = False) -> int:
        """Autotunes the kernel configuration on this Replan; returns its index."""
        h = _check_dtype(h, np.float32, "float32")
        cfg = ctypes.c_int32(-1)
        flags = ((0 if prune else PIRRT_NO_PRUNE) | (PIRRT_LOOKAHEAD if lookahead else 0) |
                 (PIRRT_TRUNCATED if truncated else 0))
        self._check(self._lib.pirrt_tune(self._h, int(root), int(goal), _ptr(h), flags, _mem_kind(h),
                                         ctypes.byref(cfg)))
        return int(cfg.value)

    def get_policy(self, device=None):
        n = self.n
        if device is not None:
            import torch
            g = torch.empty(n, dtype=torch.float32, device=device)
            p = torch.empty(n, dtype=torch.int32, device=device)
            c = torch.empty(n, dtype=torch.float32, device=device)
        else:
            g, p, c = np.empty(n, np.float32), np.empty(n, np.int32), np.empty(n, np.float32)
        self._check(self._lib.pirrt_get_policy(self._h, _ptr(g), _ptr(p), _ptr(c), _mem_kind(g, p, c)))
        return g, p, c

    def set_policy(self, g, parent, pcost) -> int:
        g = _check_dtype(g, np.float32, "float32")
        parent = _check_dtype(parent, np.int32, "int32")
        pcost = _check_dtype(pcost, np.float32, "float32")
        return self._check(self._lib.pirrt_set_policy(self._h, _ptr(g), _ptr(parent), _ptr(pcost),
                                                      _mem_kind(g, parent, pcost)))

    def snapshot_save(self) -> int:
        return self._check(self._lib.pirrt_snapshot_save(self._h))

    def snapshot_restore(self) -> int:
        return self._check(self._lib.pirrt_snapshot_restore(self._h))

    def promising_count(self, goal: int, h=None, first: int = 0, count: Optional[int] = None) -> int:
        """pirrt_promising_count: promising vertices among ids [first, first + count)."""
        h = _check_dtype(h, np.float32, "float32")
        if count is None:
            count = self.n - first
        out = ctypes.c_int64(0)
        self._check(self._lib.pirrt_promising_count(self._h, int(goal), _ptr(h), int(first), int(count),
                                                    _mem_kind(h), ctypes.byref(out)))
        return int(out.value)

    def state_size(self) -> int:
        return int(self._lib.pirrt_state_size(self._h))

    def state_save(self) -> np.ndarray:
        """pirrt_state_save into a new host byte array."""
        size = self.state_size()
        if size < 0:
            raise PirrtError(PIRRT_EINVAL, "no state blob for this handle")
        blob = np.empty(size, np.uint8)
        self._check(self._lib.pirrt_state_save(self._h, _ptr(blob), size))
        return blob

    def state_restore(self, blob) -> int:
        blob = np.ascontiguousarray(blob, np.uint8)
        return self._check(self._lib.pirrt_state_restore(self._h, _ptr(blob), int(blob.size)))

    def adjacency(self):
        ptr = np.empty(self.n + 1, np.int64)
        nbr = np.empty(max(self.nnz, 1), np.int32)
        cst = np.empty(max(self.nnz, 1), np.float32)
        self._check(self._lib.pirrt_get_adjacency(self._h, _ptr(ptr), _ptr(nbr), _ptr(cst), PIRRT_MEM_HOST))
        return ptr, nbr[: self.nnz], cst[: self.nnz]


class Batch:
    """One pirrt_batch handle: independent problems replanned together.  Vertex ids
    are local to each problem; per-vertex arrays are the problems' arrays
    concatenated in index order (``offsets`` gives where each starts)."""

    def __init__(self, stream: Optional[int] = None, device: int = -1, max_iters: int = 0,
                 vertex_capacity: int = 0, edge_capacity: int = 0, lib: Optional[ctypes.CDLL] = None):
        self._lib = lib or load()
        cfg = pirrt_config()
        self._lib.pirrt_config_init(ctypes.byref(cfg))
        cfg.vertex_capacity = vertex_capacity
        cfg.edge_capacity = edge_capacity
        cfg.hip_stream = stream or None
        cfg.max_iters = max_iters
        cfg.device = device
        h = ctypes.c_void_p()
        rc = self._lib.pirrt_batch_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_last_error(None).decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.pirrt_batch_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc: int, allow=()):
        if rc != PIRRT_OK and rc not in allow:
            raise PirrtError(rc, self._lib.pirrt_batch_last_error(self._h).decode())
        return rc

    @property
    def num_problems(self) -> int:
        return int(self._lib.pirrt_batch_num_problems(self._h))

    @property
    def n(self) -> int:
        return int(self._lib.pirrt_batch_num_vertices(self._h))

    @property
    def nnz(self) -> int:
        return int(self._lib.pirrt_batch_num_edges(self._h))

    @property
    def offsets(self) -> np.ndarray:
        return np.array([self._lib.pirrt_batch_problem_offset(self._h, i) for i in range(self.num_problems + 1)],
                        np.int64)

    def add_problem(self, row_ptr, col, cost) -> int:
        row_ptr = _check_dtype(row_ptr, np.int64, "int64")
        col = _check_dtype(col, np.int32, "int32")
        cost = _check_dtype(cost, np.float32, "float32")
        kind = _mem_kind(row_ptr, col, cost)
        idx = ctypes.c_int32(-1)
        rc = self._lib.pirrt_batch_add_problem(self._h, int(row_ptr.shape[0]) - 1, _ptr(row_ptr),
                                               _ptr(col) if len(col) else None, _ptr(cost) if len(cost) else None,
                                               kind, ctypes.byref(idx))
        self._check(rc)
        return int(idx.value)

    def problem_offset(self, problem: int) -> int:
        return int(self._lib.pirrt_batch_problem_offset(self._h, int(problem)))

    def insert(self, problems, n_new, row_ptr, col, cost) -> int:
        """pirrt_batch_insert: grows problems[k] by n_new[k] vertices; the rows of all
        blocks are concatenated in that order, in each problem's local ids."""
        problems = np.ascontiguousarray(problems, np.int32)
        n_new = np.ascontiguousarray(n_new, np.int32)
        if problems.shape != n_new.shape or problems.ndim != 1:
            raise ValueError("problems and n_new need one entry per block")
        row_ptr = _check_dtype(row_ptr, np.int64, "int64")
        col = _check_dtype(col, np.int32, "int32")
        cost = _check_dtype(cost, np.float32, "float32")
        kind = _mem_kind(row_ptr, col, cost)
        rc = self._lib.pirrt_batch_insert(self._h, int(problems.size), _ptr(problems), _ptr(n_new), _ptr(row_ptr),
                                          _ptr(col) if len(col) else None, _ptr(cost) if len(cost) else None, kind)
        return self._check(rc)

    def replan(self, roots, goals, h=None, prune: bool = True, timing: bool = False, g_out=None,
               parent_out=None, allow_not_converged: bool = False, lookahead: bool = False):
        """Replans every problem.  Returns (g, parent, per-problem stats dicts)."""
        P = self.num_problems
        roots = np.ascontiguousarray(roots, np.int32)
        goals = np.ascontiguousarray(goals, np.int32)
        if roots.shape != (P,) or goals.shape != (P,):
            raise ValueError("roots and goals need one entry per problem")
        h = _check_dtype(h, np.float32, "float32")
        n = self.n
        if g_out is None and parent_out is None and _is_device(h):
            import torch
            g_out = torch.empty(n, dtype=torch.float32, device=h.device)
            parent_out = torch.empty(n, dtype=torch.int32, device=h.device)
        if g_out is None and parent_out is None:
            g_out = np.empty(n, np.float32)
            parent_out = np.empty(n, np.int32)
        kind = _mem_kind(h, g_out, parent_out)
        flags = (0 if prune else PIRRT_NO_PRUNE) | (PIRRT_TIMING if timing else 0) | (PIRRT_LOOKAHEAD if lookahead else 0)
        st = (pirrt_stats * max(P, 1))()
        rc = self._lib.pirrt_batch_replan(self._h, _ptr(roots), _ptr(goals), _ptr(h), flags, _ptr(g_out),
                                          _ptr(parent_out), kind, ctypes.cast(st, ctypes.c_void_p))
        self._check(rc, allow=(PIRRT_ENOTCONVERGED,) if allow_not_converged else ())
        stats = [dict(st[i].as_dict(), rc=rc) for i in range(P)]
        return g_out, parent_out, stats

    def tune(self, roots, goals, h=None, prune: bool = True, lookahead: bool = False) -> int:
        """Autotunes the kernel configuration on this batch Replan; returns its index."""
        roots = np.ascontiguousarray(roots, np.int32)
        goals = np.ascontiguousarray(goals, np.int32)
        h = _check_dtype(h, np.float32, "float32")
        cfg = ctypes.c_int32(-1)
        self._check(self._lib.pirrt_batch_tune(self._h, _ptr(roots), _ptr(goals), _ptr(h),
                                               (0 if prune else PIRRT_NO_PRUNE) | (PIRRT_LOOKAHEAD if lookahead else 0),
                                               _mem_kind(h), ctypes.byref(cfg)))
        return int(cfg.value)

    def get_policy(self, device=None):
        n = self.n
        if device is not None:
            import torch
            g = torch.empty(n, dtype=torch.float32, device=device)
            p = torch.empty(n, dtype=torch.int32, device=device)
            c = torch.empty(n, dtype=torch.float32, device=device)
        else:
            g, p, c = np.empty(n, np.float32), np.empty(n, np.int32), np.empty(n, np.float32)
        self._check(self._lib.pirrt_batch_get_policy(self._h, _ptr(g), _ptr(p), _ptr(c), _mem_kind(g, p, c)))
        return g, p, c

    def snapshot_save(self) -> int:
        return self._check(self._lib.pirrt_batch_snapshot_save(self._h))

    def snapshot_restore(self) -> int:
        return self._check(self._lib.pirrt_batch_snapshot_restore(self._h))


class Rrg:
    """One pirrt_rrg handle: a scene (unit cube, sphere / box obstacles) and its
    points on the device.  `obstacles` has .d, .kind, .centre and .size arrays (or
    is None for free space)."""

    def __init__(self, d: int, obstacles=None, stream: Optional[int] = None, device: int = -1,
                 point_capacity: int = 0, lib: Optional[ctypes.CDLL] = None):
        self._lib = lib or load()
        self.d = int(d)
        m = 0 if obstacles is None else len(obstacles.kind)
        self._kind = np.ascontiguousarray(obstacles.kind if m else np.zeros(1), np.int32)
        self._centre = np.ascontiguousarray(obstacles.centre if m else np.zeros((1, d)), np.float64)
        self._size = np.ascontiguousarray(obstacles.size if m else np.zeros((1, d)), np.float64)
        cfg = pirrt_rrg_config()
        cfg.d = self.d
        cfg.n_obstacles = m
        cfg.kind = self._kind.ctypes.data
        cfg.centre = self._centre.ctypes.data
        cfg.size = self._size.ctypes.data
        cfg.point_capacity = point_capacity
        cfg.hip_stream = stream or None
        cfg.device = device
        h = ctypes.c_void_p()
        rc = self._lib.pirrt_rrg_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_rrg_last_error(None).decode())
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.pirrt_rrg_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc: int):
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_rrg_last_error(self._h).decode())
        return rc

    @property
    def n(self) -> int:
        return int(self._lib.pirrt_rrg_num_points(self._h))

    def add_points(self, pts) -> int:
        pts = _check_dtype(pts, np.float64, "float64")
        count = int(pts.shape[0]) if pts.ndim > 1 else int(pts.shape[0]) // self.d
        return self._check(self._lib.pirrt_rrg_add_points(self._h, count, _ptr(pts), _mem_kind(pts)))

    def sample(self, seed: int, stream: int, counter: int, count: int) -> int:
        """Appends `count` free samples; returns the next counter."""
        c = ctypes.c_uint64(counter)
        self._check(self._lib.pirrt_rrg_sample(self._h, int(seed), int(stream), ctypes.byref(c), int(count)))
        return int(c.value)

    def sample_learned(self, net: "Mlp", enc, seed: int, stream: int, counter: int, n_candidates: int,
                       count: int) -> int:
        """Appends the `count` best-scored of n_candidates free candidates; returns
        the next counter."""
        enc = np.ascontiguousarray(enc, np.float32)
        c = ctypes.c_uint64(counter)
        self._check(self._lib.pirrt_rrg_sample_learned(self._h, net._h, enc.ctypes.data if len(enc) else None,
                                                       len(enc), int(seed), int(stream), ctypes.byref(c),
                                                       int(n_candidates), int(count)))
        return int(c.value)

    def points(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.n - first if count is None else count
        out = np.empty((max(count, 0), self.d), np.float64)
        self._check(self._lib.pirrt_rrg_get_points(self._h, first, count, _ptr(out), PIRRT_MEM_HOST))
        return out

    def rows(self, n_old: int, radius: float, device=None, capacity: Optional[int] = None):
        """Forward rows (row_ptr, col, cost) of points n_old .. n-1, on the host, or as
        device tensors with `device` (one radius search when `capacity` entries suffice,
        default 128 a row)."""
        if device is not None:
            import torch
            rows = self.n - n_old
            cap = int(capacity if capacity is not None else max(rows, 1) * 128)
            nnz = ctypes.c_int64(0)
            rp = torch.empty(rows + 1, dtype=torch.int64, device=device)
            for _ in range(2):
                col = torch.empty(max(cap, 1), dtype=torch.int32, device=device)
                cost = torch.empty(max(cap, 1), dtype=torch.float32, device=device)
                rc = self._lib.pirrt_rrg_rows(self._h, n_old, radius, _ptr(rp), _ptr(col), _ptr(cost), cap,
                                              ctypes.byref(nnz), PIRRT_MEM_DEVICE)
                if rc == PIRRT_OK:
                    m = int(nnz.value)
                    return rp, col[:m], cost[:m]
                if rc != PIRRT_EINVAL or nnz.value <= cap:
                    self._check(rc)
                cap = int(nnz.value)
            self._check(rc)
        nnz = ctypes.c_int64(0)
        rp = np.empty(self.n - n_old + 1, np.int64)
        rc = self._lib.pirrt_rrg_rows(self._h, n_old, radius, _ptr(rp), None, None, 0, ctypes.byref(nnz),
                                      PIRRT_MEM_HOST)
        if rc not in (PIRRT_OK, PIRRT_EINVAL) or (rc == PIRRT_EINVAL and nnz.value == 0 and self.n > n_old):
            self._check(rc)
        m = int(nnz.value)
        col = np.empty(max(m, 1), np.int32)
        cost = np.empty(max(m, 1), np.float32)
        self._check(self._lib.pirrt_rrg_rows(self._h, n_old, radius, _ptr(rp), _ptr(col), _ptr(cost), m,
                                             ctypes.byref(nnz), PIRRT_MEM_HOST))
        return rp, col[:m], cost[:m]

    def connect(self, n_old: int, radius: float, graph: "Graph") -> int:
        return self._check(self._lib.pirrt_rrg_connect(self._h, n_old, radius, graph.handle))

    def connect_problem(self, radius: float, batch: "Batch") -> int:
        idx = ctypes.c_int32(-1)
        self._check(self._lib.pirrt_rrg_connect_problem(self._h, radius, batch._h, ctypes.byref(idx)))
        return int(idx.value)

    def heuristic(self, goal: int, out=None):
        out = np.empty(self.n, np.float32) if out is None else out
        self._check(self._lib.pirrt_rrg_heuristic(self._h, goal, _ptr(out), _mem_kind(out)))
        return out


class Mlp:
    """One pirrt_mlp handle (the learned proposal's network).  Parameters travel as
    one float32 array in the layout of include/pirrt.h (W1 [288 x 256], b1, W2, b2,
    w3, b3)."""

    def __init__(self, in_dim: int, max_batch: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, stream: Optional[int] = None, device: int = -1, lib: Optional[ctypes.CDLL] = None):
        self._lib = lib or load()
        cfg = pirrt_mlp_config(in_dim, max_batch, lr, beta1, beta2, eps, stream or None, device)
        h = ctypes.c_void_p()
        rc = self._lib.pirrt_mlp_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_mlp_last_error(None).decode())
        self._h = h
        self.in_dim = in_dim
        self.num_params = int(self._lib.pirrt_mlp_num_params())

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.pirrt_mlp_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc: int):
        if rc != PIRRT_OK:
            raise PirrtError(rc, self._lib.pirrt_mlp_last_error(self._h).decode())
        return rc

    def set_params(self, params) -> int:
        params = _check_dtype(params, np.float32, "float32")
        return self._check(self._lib.pirrt_mlp_set_params(self._h, _ptr(params), _mem_kind(params)))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, np.float32)
        self._check(self._lib.pirrt_mlp_get_params(self._h, _ptr(out), PIRRT_MEM_HOST))
        return out

    def forward(self, x, out=None):
        x = _check_dtype(x, np.float32, "float32")
        B = int(x.shape[0])
        if out is None:
            if _is_device(x):
                import torch
                out = torch.empty(B, dtype=torch.float32, device=x.device)
            else:
                out = np.empty(B, np.float32)
        self._check(self._lib.pirrt_mlp_forward(self._h, B, _ptr(x), _ptr(out), _mem_kind(x, out)))
        return out

    def forward_noalloc(self, x, out):
        """pirrt_mlp_forward_noalloc: device tensors only; enqueued on the handle's
        stream without waiting (the caller synchronises)."""
        x = _check_dtype(x, np.float32, "float32")
        out = _check_dtype(out, np.float32, "float32")
        if not (_is_device(x) and _is_device(out)):
            raise ValueError("forward_noalloc takes device tensors")
        return self._check(self._lib.pirrt_mlp_forward_noalloc(self._h, int(x.shape[0]), _ptr(x), _ptr(out)))

    def gradients(self, x, y):
        x = _check_dtype(x, np.float32, "float32")
        y = _check_dtype(y, np.float32, "float32")
        g = np.empty(self.num_params, np.float32)
        loss = ctypes.c_float(0.0)
        if _is_device(x):
            import torch
            gd = torch.empty(self.num_params, dtype=torch.float32, device=x.device)
            self._check(self._lib.pirrt_mlp_gradients(self._h, int(x.shape[0]), _ptr(x), _ptr(y), _ptr(gd),
                                                      ctypes.byref(loss), PIRRT_MEM_DEVICE))
            return float(loss.value), gd.cpu().numpy()
        self._check(self._lib.pirrt_mlp_gradients(self._h, int(x.shape[0]), _ptr(x), _ptr(y), _ptr(g),
                                                  ctypes.byref(loss), PIRRT_MEM_HOST))
        return float(loss.value), g

    def train_step(self, x, y) -> float:
        x = _check_dtype(x, np.float32, "float32")
        y = _check_dtype(y, np.float32, "float32")
        loss = ctypes.c_float(0.0)
        self._check(self._lib.pirrt_mlp_train_step(self._h, int(x.shape[0]), _ptr(x), _ptr(y), ctypes.byref(loss),
                                                   _mem_kind(x, y)))
        return float(loss.value)


def pirrt_strerror(code: int) -> str:
    return _strerror(code)
