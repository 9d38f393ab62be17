"""The learned sampling proposal around the library's network (pirrt_mlp_*): its
input encoding, the labels it learns from, and the training loop.  Host
orchestration only: the graphs, Replans and every forward and backward pass run in
the library.

- Input: a sample's coordinates, then the scene's spheres as (centre, radius) in
  order, zero-padded to 40 slots (for 6D, 6 + 280 = 286 values).
- Label (not in the paper): a vertex is positive when a path through it is within 5%
  of the best, g_r(v) + g_t(v) <= 1.05 g_r(goal) summed in binary64, with g_r from a
  Replan rooted at x_init and g_t from one rooted at x_goal, both without pruning, on
  the same converged graph.
- Training: mean BCE-with-logits with Adam (pirrt_mlp_train_step) on batches drawn
  without replacement from positive-balanced per-layout samples.
"""
from __future__ import annotations

import time
from typing import List, Optional, Tuple

import numpy as np

from .binding import Graph, Mlp, Rrg
from .planner import radius, root_goal

SLOTS = 40  # sphere slots of the encoding
K_IN = 288  # the network's padded input width


def sphere_encoding(obstacles, slots: int = SLOTS) -> np.ndarray:
    """The spheres (kind 0) of a scene as (centre, radius), zero-padded to `slots`."""
    d = int(obstacles.d)
    enc = np.zeros(slots * (d + 1), np.float32)
    k = 0
    for o in range(len(obstacles.kind)):
        if obstacles.kind[o] == 0 and k < slots:
            enc[k * (d + 1):k * (d + 1) + d] = obstacles.centre[o]
            enc[k * (d + 1) + d] = obstacles.size[o, 0]
            k += 1
    return enc


def init_params(in_dim: int, seed: int) -> np.ndarray:
    """He-scaled normal weights, zero biases, in the library's parameter layout
    (W1 [288 x 256] with rows past in_dim zero, b1, W2 [256 x 256], b2, w3, b3)."""
    rng = np.random.default_rng(seed)
    h = 256
    p = np.zeros(K_IN * h + h + h * h + h + h + 1, np.float32)
    p[:in_dim * h] = (rng.standard_normal((in_dim, h)) * np.sqrt(2.0 / in_dim)).ravel()
    o = K_IN * h + h
    p[o:o + h * h] = rng.standard_normal(h * h) * np.sqrt(2.0 / h)
    o += h * h + h
    p[o:o + h] = rng.standard_normal(h) * np.sqrt(1.0 / h)
    return p


def labels(graph: Graph) -> np.ndarray:
    """Binary labels of every vertex of a graph (root 0, goal 1): near-optimal-path
    membership from two Replans without pruning."""
    g_r, _, _ = graph.replan(0, 1, None, False)
    g_t, _, _ = graph.replan(1, 0, None, False)
    best = float(g_r[1])
    tot = g_r.astype(np.float64) + g_t.astype(np.float64)
    return (np.isfinite(tot) & (tot <= 1.05 * best)).astype(np.float32)


def layout_samples(d: int, obstacles, seed: int, n: int, per_layout: int, rng: np.random.Generator,
                   stream=None, device: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Grows one layout's graph to n vertices at once (uniform samples of `seed`),
    labels it and keeps per_layout vertices, half positive where there are enough.
    Returns (features [k x (d + 40 (d + 1))], labels [k])."""
    R = Rrg(d, obstacles, stream=stream, point_capacity=n, device=device)
    R.add_points(root_goal(d))
    R.sample(seed, 0, 0, n - 2)
    G = Graph(stream=stream, vertex_capacity=n, device=device)
    R.connect(0, radius(n, d), G)
    lab = labels(G)
    pos = np.nonzero(lab > 0)[0]
    neg = np.nonzero(lab == 0)[0]
    k_pos = min(len(pos), per_layout // 2)
    k_neg = min(len(neg), per_layout - k_pos)
    pick = np.concatenate([rng.choice(pos, k_pos, replace=False), rng.choice(neg, k_neg, replace=False)])
    pts = R.points()[pick].astype(np.float32)
    enc = sphere_encoding(obstacles)
    return np.concatenate([pts, np.broadcast_to(enc, (len(pick), len(enc)))], axis=1), lab[pick]


def train(net: Mlp, X, Y, epochs: int, batch: int = 4096, seed: int = 0) -> Tuple[List[float], float]:
    """Adam steps over `epochs` passes of (X, Y) (device tensors) in shuffled batches;
    returns the per-step losses and the seconds taken."""
    import torch
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    losses: List[float] = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(epochs):
        order = torch.randperm(len(Y), device=X.device, generator=g)
        for i in range(0, len(Y) - batch + 1, batch):
            idx = order[i:i + batch]
            losses.append(net.train_step(X[idx].contiguous(), Y[idx].contiguous()))
    torch.cuda.synchronize()
    return losses, time.perf_counter() - t0


def build_and_train(d: int, make_obstacles, layout_seeds, n: int, per_layout: int, epochs: int,
                    stream=None, device: int = 0, batch: int = 4096, init_seed: int = 11,
                    log=None) -> Tuple[Mlp, dict]:
    """Training data from the given layouts (make_obstacles(seed) gives a scene, its
    samples use seed + 1), then a network trained on the device.  Returns the network
    and a record (sample count, positive share, data and training seconds, losses)."""
    import torch
    dev = torch.device("cuda", device)
    rng = np.random.default_rng(7)
    xs, ys = [], []
    t0 = time.perf_counter()
    for i, s in enumerate(layout_seeds):
        x, y = layout_samples(d, make_obstacles(s), s + 1, n, per_layout, rng, stream=stream, device=device)
        xs.append(x)
        ys.append(y)
        if log and (i + 1) % 100 == 0:
            log("training data: %d of %d layouts (%.1f s)" % (i + 1, len(layout_seeds), time.perf_counter() - t0))
    X = torch.from_numpy(np.ascontiguousarray(np.concatenate(xs), np.float32)).to(dev)
    Y = torch.from_numpy(np.concatenate(ys)).to(dev)
    data_s = time.perf_counter() - t0
    net = Mlp(X.shape[1], 8192, lr=1e-3, stream=stream, device=device)
    net.set_params(init_params(X.shape[1], init_seed))
    losses, train_s = train(net, X, Y, epochs, batch)
    rec = {"layouts": len(layout_seeds), "samples": int(len(Y)), "positive_share": float(Y.mean()),
           "data_seconds": data_s, "train_seconds": train_s, "steps": len(losses), "batch": batch,
           "loss_first": float(np.mean(losses[:20])) if losses else None,
           "loss_last": float(np.mean(losses[-20:])) if losses else None}
    return net, rec


def time_to_cost(history, target: float) -> Optional[float]:
    """First wall time in a planner history at which g(goal) <= target (None if never)."""
    for r in history:
        if r["cost"] <= target:
            return r["seconds"]
    return None
