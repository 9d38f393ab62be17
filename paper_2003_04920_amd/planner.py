"""Planners around Replan: host orchestration of the library's entry points only.

Every step runs in the library (sampling, radius neighbours and segment tests,
insertion-time policy, the replan test, Replan); this module only decides what to call
next, the way Alg. 1 and Alg. 3 of "GPU Parallelization of Policy Iteration RRT#"
(arXiv 2003.04920) arrange Extend and Replan:

- ``Planner``: Batched-Extension PI-RRT# (BERRT#, Alg. 3).  Each batch extends the
  graph by S samples (Extend, Sec. III) and replans when the batch added a promising
  vertex (the test |B'| > |B|, ``pirrt_promising_count``), or after every batch.  With
  S = 1 it is PI-RRT# itself (Alg. 1).  With a network (the learned proposal), half of
  every batch is the best-scored of a set of uniform candidates and half uniform.
- ``plan_concurrent``: exploration concurrent with exploitation (the asynchronous
  scheme of Sec. VII): an explorer thread samples and builds the rows of each batch on
  one stream while the exploiter inserts every queued batch and replans on another.

Vertex 0 is x_init = (0.05)^d and vertex 1 is x_goal = (0.95)^d; the radius is
r = gamma (ln n / n)^(1/d) at the vertex count after the batch; h is the Euclidean
distance to x_goal rounded to binary32 (the library computes it).
"""
from __future__ import annotations

import math
import queue
import threading
import time
from typing import Callable, List, Optional

import numpy as np

from .binding import Graph, Mlp, Rrg


def radius(n: int, d: int, gamma: float = 1.0) -> float:
    """Connection radius gamma (ln n / n)^(1/d) (the RRG's shrinking neighbourhood)."""
    n = max(n, 2)
    return gamma * (math.log(n) / n) ** (1.0 / d)


def root_goal(d: int) -> np.ndarray:
    return np.stack([np.full(d, 0.05), np.full(d, 0.95)])


class Planner:
    """BERRT# (Alg. 3) on one device.

    d, obstacles: the scene (obstacles as for ``Rrg``); seed: sample seed (uniform
    samples use stream 0 of it, learned candidates stream 1); capacity: vertices to
    reserve; trigger: replan only when a batch adds a promising vertex (else after every
    batch); net / enc: the learned proposal's network and the scene's encoding;
    candidates: candidates scored per learned draw.  Device buffers for h, g and the
    parents are torch tensors on ``device`` (PyTorch provides memory and streams only).
    """

    def __init__(self, d: int, obstacles, seed: int, capacity: int, stream=None, device: int = 0,
                 trigger: bool = True, net: Optional[Mlp] = None, enc=None, candidates: int = 8192,
                 gamma: float = 1.0):
        import torch
        self._torch = torch
        self.d, self.seed, self.gamma = int(d), int(seed), float(gamma)
        self.trigger = bool(trigger)
        self.net, self.enc, self.candidates = net, enc, int(candidates)
        self.dev = torch.device("cuda", device)
        self.stream = stream
        sid = stream.cuda_stream if stream is not None else None
        self.rrg = Rrg(d, obstacles, stream=sid, point_capacity=capacity, device=device)
        self.rrg.add_points(root_goal(d))
        self.graph = Graph(stream=sid, vertex_capacity=capacity, device=device)
        self.rrg.connect(0, radius(2, d, gamma), self.graph)
        self.counter_uniform = 0
        self.counter_learned = 0
        self.replans = 0
        self.history: List[dict] = []
        self.goal_cost = float(self.graph.get_policy()[0][1])

    @property
    def n(self) -> int:
        return self.rrg.n

    def _h(self):
        n = self.n
        return self.rrg.heuristic(1, out=self._torch.empty(n, dtype=self._torch.float32, device=self.dev))

    def extend(self, S: int) -> int:
        """Extend by S samples (Alg. 3's inner loop as one batch): draws, radius search
        at the new vertex count, insertion with the insertion-time policy.  Returns the
        first new vertex id."""
        n_old = self.n
        if self.net is not None:
            k = S // 2
            if k:
                self.counter_learned = self.rrg.sample_learned(self.net, self.enc, self.seed, 1,
                                                               self.counter_learned, self.candidates, k)
            self.counter_uniform = self.rrg.sample(self.seed, 0, self.counter_uniform, S - k)
        else:
            self.counter_uniform = self.rrg.sample(self.seed, 0, self.counter_uniform, S)
        self.rrg.connect(n_old, radius(self.n, self.d, self.gamma), self.graph)
        return n_old

    def replan(self, h=None) -> dict:
        h = self._h() if h is None else h
        n = self.n
        g = self._torch.empty(n, dtype=self._torch.float32, device=self.dev)
        p = self._torch.empty(n, dtype=self._torch.int32, device=self.dev)
        _, _, st = self.graph.replan(0, 1, h, True, g_out=g, parent_out=p)
        self.replans += 1
        self.goal_cost = float(g[1].item())
        return st

    def step(self, S: int) -> dict:
        """One batch of Alg. 3: extend by S, then Replan if |B'| > |B| (or always
        without the trigger)."""
        n_old = self.extend(S)
        h = self._h()
        promising = self.graph.promising_count(1, h, n_old, self.n - n_old)
        due = promising > 0 or not self.trigger
        if due:
            self.replan(h)
        rec = {"n": self.n, "promising_new": promising, "replanned": due, "cost": self.goal_cost}
        self.history.append(rec)
        return rec

    def run(self, N: int, S: int, on_batch: Optional[Callable[[dict], None]] = None) -> List[dict]:
        """Grows to N free samples in batches of S (the last batch may be smaller);
        records the wall time and g(goal) (the cost of the best path found, +inf while
        the goal is unreached) after every batch."""
        t0 = time.perf_counter()
        while self.n - 2 < N:
            rec = self.step(min(S, N - (self.n - 2)))
            rec["seconds"] = time.perf_counter() - t0
            if on_batch:
                on_batch(rec)
        return self.history


def plan_concurrent(d: int, obstacles, seed: int, N: int, S: int, device: int = 0, gamma: float = 1.0,
                    keep_start: bool = False):
    """Exploration concurrent with exploitation (Sec. VII's asynchronous scheme).

    An explorer thread draws each batch and builds its forward rows on its own stream
    and queues them; the exploiter (the calling thread) inserts every queued batch on a
    second stream and replans once per drained queue, so later radius searches overlap
    earlier Replans.  The last Replan runs after every batch was inserted.  Returns
    (graph, rrg, replans, start) where start is, with keep_start, the policy (g,
    parent, pcost) the last Replan started from (so that a checker can replay it), else
    None."""
    import torch
    dev = torch.device("cuda", device)
    sa, sb = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    R = Rrg(d, obstacles, stream=sa.cuda_stream, point_capacity=N + 2, device=device)
    R.add_points(root_goal(d))
    G = Graph(stream=sb.cuda_stream, vertex_capacity=N + 2, device=device)
    rp0, c0, w0 = R.rows(0, radius(2, d, gamma), device=dev)
    sa.synchronize()
    with torch.cuda.stream(sb):
        G.insert_batch(rp0, c0, w0)
    q: "queue.Queue" = queue.Queue()
    err: List[BaseException] = []

    def explorer():
        try:
            with torch.cuda.stream(sa):
                counter, n_old = 0, 2
                while R.n - 2 < N:
                    counter = R.sample(seed, 0, counter, min(S, N - (R.n - 2)))
                    n = R.n
                    rp, col, cost = R.rows(n_old, radius(n, d, gamma), device=dev)
                    h = R.heuristic(1, out=torch.empty(n, dtype=torch.float32, device=dev))
                    sa.synchronize()
                    q.put((rp, col, cost, h))
                    n_old = n
        except BaseException as e:  # re-raised by the exploiter
            err.append(e)
        q.put(None)

    replans, done, before = 0, False, None
    th = threading.Thread(target=explorer)
    th.start()
    with torch.cuda.stream(sb):
        while not done:
            items = [q.get()]
            while True:
                try:
                    items.append(q.get_nowait())
                except queue.Empty:
                    break
            h = None
            for it in items:
                if it is None:
                    done = True
                    continue
                rp, col, cost, h = it
                G.insert_batch(rp, col, cost)
            if h is not None:
                if keep_start:
                    before = G.get_policy()
                G.replan(0, 1, h, True)
                replans += 1
    th.join()
    torch.cuda.synchronize()
    if err:
        raise err[0]
    return G, R, replans, before
