"""Seeded synthetic planning workloads (inputs only).

Builds the random geometric graphs (RRG) that PI-RRT#'s exploration phase grows
(Sec. III; Alg. 1 and Alg. 3), for the five workload shapes the planner is
measured on.  The output of this module is plain data -- sample points, the
forward CSR rows of every inserted batch (each new vertex lists its lower-index
neighbours within radius r whose segment is collision free, with the FP32 rounding
of the FP64 Euclidean length as cost), and an FP32 Euclidean heuristic to the
goal.  It contains none of policy evaluation / improvement, so both the oracle
and the GPU path consume it.

Conventions (chosen here; the paper's 2D polygon scene is unpublished):
  * vertex 0 = x_init, vertex 1 = x_goal (Alg. 1 starts from V = {x_init, x_goal});
    the first batch holds them plus its samples, in that order.
  * d-dimensional unit cube; x_init = (0.05,)*d, x_goal = (0.95,)*d.
  * obstacles: spheres (centre uniform, radius U(0.05, 0.15)) or axis-aligned
    boxes (centre uniform, side U(0.05, 0.2) drawn per axis); an obstacle that
    would cover x_init or x_goal is drawn again.
  * samples are uniform and rejected when inside (or on) an obstacle; draws
    continue until the stated number of free samples is reached.
  * r = (ln n / n)^(1/d) with n the vertex count after the batch.
  * randomness: numpy's Philox counter-based generator keyed by the seed.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rrg_geom.c")
_LIB = os.path.join(_HERE, "librrg_geom.so")
_lib = None


def build_geom(force: bool = False) -> str:
    """Compiles the geometry helper with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Rows(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)), ("cost", ctypes.POINTER(ctypes.c_float))]


def _geom():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_geom()
        lib = ctypes.CDLL(_LIB)
        lib.rrg_build_rows.restype = ctypes.c_int
        lib.rrg_build_rows.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Rows)]
        lib.rrg_free_rows.restype = None
        lib.rrg_free_rows.argtypes = [ctypes.POINTER(_Rows)]
        lib.rrg_point_blocked.restype = ctypes.c_int
        lib.rrg_point_blocked.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _threads() -> int:
    try:
        return max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1))
    except ValueError:
        return max(1, min(16, os.cpu_count() or 1))


@dataclass
class Obstacles:
    d: int
    kind: np.ndarray     # int32[k]: 0 sphere, 1 box
    centre: np.ndarray   # float64[k, d]
    size: np.ndarray     # float64[k, d]: sphere radius in column 0; box half-sides

    def blocked(self, x: np.ndarray) -> np.ndarray:
        """Boolean mask of points inside (or on) any obstacle (closed sets)."""
        x = np.atleast_2d(x)
        out = np.zeros(len(x), dtype=bool)
        for o in range(len(self.kind)):
            c = self.centre[o]
            if self.kind[o] == 0:
                out |= ((x - c) ** 2).sum(axis=1) <= self.size[o, 0] ** 2
            else:
                out |= (np.abs(x - c) <= self.size[o]).all(axis=1)
        return out


@dataclass
class Batch:
    n_old: int
    n_new: int
    row_ptr: np.ndarray  # int64[n_new + 1]
    col: np.ndarray      # int32[nnz]; col[j] < n_old + row
    cost: np.ndarray     # float32[nnz], > 0
    radius: float

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


@dataclass
class Workload:
    name: str
    d: int
    points: np.ndarray          # float64[n, d]
    obstacles: Obstacles
    batches: List[Batch] = field(default_factory=list)
    root: int = 0
    goal: int = 1

    @property
    def n(self) -> int:
        return len(self.points)

    def heuristic(self, n: Optional[int] = None) -> np.ndarray:
        """FP32 rounding of the FP64 Euclidean distance to the goal (admissible)."""
        pts = self.points if n is None else self.points[:n]
        return np.sqrt(((pts - self.points[self.goal]) ** 2).sum(axis=1)).astype(np.float32)

    @property
    def nnz(self) -> int:
        return sum(b.nnz for b in self.batches)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=int(seed)))


def make_obstacles(d: int, count: int, kinds: str, seed: int) -> Obstacles:
    """`kinds` is 'sphere', 'box' or 'mixed' (each obstacle 50/50)."""
    rng = _rng(seed)
    start = np.full(d, 0.05)
    goal = np.full(d, 0.95)
    kind = np.zeros(count, np.int32)
    centre = np.zeros((count, d))
    size = np.zeros((count, d))
    for o in range(count):
        while True:
            if kinds == "sphere":
                k = 0
            elif kinds == "box":
                k = 1
            else:
                k = int(rng.random() < 0.5)
            c = rng.random(d)
            if k == 0:
                s = np.zeros(d)
                s[0] = 0.05 + 0.10 * rng.random()
                bad = any(((p - c) ** 2).sum() <= s[0] ** 2 for p in (start, goal))
            else:
                s = 0.5 * (0.05 + 0.15 * rng.random(d))
                bad = any((np.abs(p - c) <= s).all() for p in (start, goal))
            if not bad:
                break
        kind[o], centre[o], size[o] = k, c, s
    return Obstacles(d, kind, centre, size)


def sample_free(rng: np.random.Generator, obs: Obstacles, count: int) -> np.ndarray:
    """`count` uniform free samples in draw order (rejection sampling)."""
    out = np.zeros((count, obs.d))
    got = 0
    while got < count:
        want = max(1024, int((count - got) * 1.3))
        x = rng.random((want, obs.d))
        x = x[~obs.blocked(x)]
        take = min(len(x), count - got)
        out[got:got + take] = x[:take]
        got += take
    return out


def radius(n: int, d: int, gamma: float = 1.0) -> float:
    """Connection radius gamma * (ln n / n)^(1/d)."""
    return gamma * (math.log(n) / n) ** (1.0 / d)


def build_rows(points: np.ndarray, n_old: int, n_new: int, r: float, obs: Obstacles,
               nthreads: Optional[int] = None) -> Batch:
    """Forward rows of vertices n_old .. n_old+n_new-1 (neighbours u < v, ascending)."""
    lib = _geom()
    pts = np.ascontiguousarray(points[: n_old + n_new], dtype=np.float64)
    kind = np.ascontiguousarray(obs.kind, dtype=np.int32)
    centre = np.ascontiguousarray(obs.centre, dtype=np.float64)
    size = np.ascontiguousarray(obs.size, dtype=np.float64)
    rows = _Rows()
    rc = lib.rrg_build_rows(obs.d, n_old, n_new, pts.ctypes.data, r, len(kind),
                            kind.ctypes.data if len(kind) else None,
                            centre.ctypes.data if len(kind) else None,
                            size.ctypes.data if len(kind) else None,
                            nthreads or _threads(), ctypes.byref(rows))
    if rc != 0:
        raise RuntimeError("rrg_build_rows failed (%d)" % rc)
    try:
        nnz = int(rows.nnz)
        row_ptr = np.ctypeslib.as_array(rows.row_ptr, shape=(n_new + 1,)).copy()
        col = np.ctypeslib.as_array(rows.col, shape=(max(nnz, 1),))[:nnz].copy()
        cost = np.ctypeslib.as_array(rows.cost, shape=(max(nnz, 1),))[:nnz].copy()
    finally:
        lib.rrg_free_rows(ctypes.byref(rows))
    return Batch(n_old, n_new, row_ptr, col, cost, r)


def grow(name: str, d: int, obs: Obstacles, sample_seed: int, batch_sizes: List[int],
         gamma: float = 1.0, nthreads: Optional[int] = None) -> Workload:
    """Draws the samples and builds one forward-row batch per entry of `batch_sizes`
    (free-sample counts; the first batch also holds x_init and x_goal)."""
    rng = _rng(sample_seed)
    total = sum(batch_sizes)
    samples = sample_free(rng, obs, total)
    pts = np.concatenate([np.full((1, d), 0.05), np.full((1, d), 0.95), samples], axis=0)
    wl = Workload(name, d, pts, obs)
    n_old = 0
    for i, s in enumerate(batch_sizes):
        n_new = s + (2 if i == 0 else 0)
        n = n_old + n_new
        wl.batches.append(build_rows(pts, n_old, n_new, radius(n, d, gamma), obs, nthreads))
        n_old = n
    return wl


# ---------------------------------------------------------------------------
# The workload shapes.  Seeds: layout seed, sample seed.
# ---------------------------------------------------------------------------

def plain_2d(samples: int = 2000, seed: int = 0) -> Workload:
    """2D unit square, 8 boxes, 2,000 free samples, one batch (the small case)."""
    obs = make_obstacles(2, 8, "box", seed)
    return grow("plain-2d-2k", 2, obs, seed + 1, [samples])


def batched_6d(batches: int = 100, batch: int = 1000, seed: int = 100) -> Workload:
    """6D unit cube, 40 spheres, `batches` x `batch` free samples (r at the current n)."""
    obs = make_obstacles(6, 40, "sphere", seed)
    return grow("berrt-6d-%dx%d" % (batches, batch), 6, obs, seed + 1, [batch] * batches)


def plain_6d(samples: int = 1_000_000, extra: int = 10_000, seed: int = 200,
             nthreads: Optional[int] = None) -> Workload:
    """6D unit cube, 40 spheres, `samples` free samples in one batch, then `extra`."""
    obs = make_obstacles(6, 40, "sphere", seed)
    sizes = [samples] + ([extra] if extra else [])
    return grow("plain-6d-%d" % samples, 6, obs, seed + 1, sizes, nthreads=nthreads)


def multi_problem(index: int, base_seed: int = 1000, n_min: int = 5000, n_max: int = 200_000,
                  samples: Optional[int] = None) -> Workload:
    """Problem `index` of the multi-graph set: d in {2,3,4,6,8}, n log-uniform in
    [n_min, n_max], 10-40 obstacles (each a sphere or a box, 50/50)."""
    rng = _rng(base_seed + index)
    d = int(rng.choice([2, 3, 4, 6, 8]))
    n = int(round(math.exp(math.log(n_min) + rng.random() * (math.log(n_max) - math.log(n_min)))))
    k = int(rng.integers(10, 41))
    obs = make_obstacles(d, k, "mixed", base_seed + 100_000 + index)
    return grow("multi-%d" % index, d, obs, base_seed + 200_000 + index,
                [samples if samples is not None else max(1, n - 2)])


@dataclass
class ProblemSpec:
    """A multi-graph problem without its samples: the device samples them (Philox,
    stream 0 under `sample_seed`) after x_init = (0.05)^d and x_goal = (0.95)^d."""
    index: int
    d: int
    n: int                 # vertices including x_init and x_goal
    obstacles: Obstacles
    sample_seed: int

    @property
    def radius(self) -> float:
        return radius(self.n, self.d)


def multi_problem_spec(index: int, base_seed: int = 1000, n_min: int = 5000,
                       n_max: int = 200_000) -> ProblemSpec:
    """Problem `index` of the multi-graph set with the same d, n and obstacles as
    multi_problem(index, ...)."""
    rng = _rng(base_seed + index)
    d = int(rng.choice([2, 3, 4, 6, 8]))
    n = int(round(math.exp(math.log(n_min) + rng.random() * (math.log(n_max) - math.log(n_min)))))
    k = int(rng.integers(10, 41))
    obs = make_obstacles(d, k, "mixed", base_seed + 100_000 + index)
    return ProblemSpec(index, d, max(n, 3), obs, base_seed + 200_000 + index)


def sphere_encoding(obs: Obstacles, slots: int = 40) -> np.ndarray:
    """Input format of the learned proposal: the spheres' (centre, radius) in order,
    zero-padded to `slots` entries of d + 1 values (binary32)."""
    d = obs.d
    enc = np.zeros(slots * (d + 1), np.float32)
    k = 0
    for o in range(len(obs.kind)):
        if obs.kind[o] == 0 and k < slots:
            enc[k * (d + 1):k * (d + 1) + d] = obs.centre[o]
            enc[k * (d + 1) + d] = obs.size[o, 0]
            k += 1
    return enc


def path_graph(n: int, costs: np.ndarray) -> Batch:
    """A path 0-1-2-...-(n-1); costs[i] is the cost of edge (i, i+1)."""
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[2:] = np.arange(1, n)
    col = np.arange(0, n - 1, dtype=np.int32)
    return Batch(0, n, row_ptr, col, np.asarray(costs, np.float32), 0.0)


def from_edges(n: int, edges, n_old: int = 0) -> Batch:
    """Forward rows for vertices n_old..n-1 from an undirected edge list
    [(a, b, cost)] in which every edge has its higher endpoint >= n_old."""
    rows = [[] for _ in range(n - n_old)]
    for a, b, c in edges:
        lo, hi = (a, b) if a < b else (b, a)
        if hi < n_old or lo == hi:
            raise ValueError("edge (%d,%d) is not a forward edge of this batch" % (a, b))
        rows[hi - n_old].append((lo, np.float32(c)))
    row_ptr = np.zeros(n - n_old + 1, np.int64)
    col, cost = [], []
    for i, r in enumerate(rows):
        r.sort(key=lambda t: t[0])  # stable: parallel edges keep their given order
        row_ptr[i + 1] = row_ptr[i] + len(r)
        col += [u for u, _ in r]
        cost += [c for _, c in r]
    return Batch(n_old, n - n_old, row_ptr, np.asarray(col, np.int32), np.asarray(cost, np.float32), 0.0)
