"""ORACLE (test infrastructure only): the learned sampling proposal's network in
plain numpy -- the statement the device kernels are checked against.

Network: features f (the sample's d coordinates, then the obstacle encoding, zero-
padded to K = 288 columns) -> 256 -> 256 -> 1 logit, ReLU after the two hidden
layers.  Arithmetic contract (what the device does, stated step by step):

  * parameters are kept in binary32 (the master copy); every matrix product uses
    their bfloat16 rounding (round to nearest even) and bfloat16 activations, with
    exact products and binary32-or-wider accumulation;
  * X  = bf16(f)
    Z1 = X @ bf16(W1) + b1,          A1 = bf16(relu(Z1))
    Z2 = A1 @ bf16(W2) + b2,         A2 = bf16(relu(Z2))
    z  = A2 @ bf16(w3) + b3
  * loss = mean over the batch of BCE-with-logits(z, y)
         = mean(max(z, 0) - z*y + log(1 + exp(-|z|)));
  * backward (dz = (sigmoid(z) - y) / B):
      gw3 = A2^T dz,  gb3 = sum dz
      dZ2 = bf16((dz w3^T) * [Z2 > 0]),  gW2 = A1^T dZ2,  gb2 = column sums of dZ2
      dZ1 = bf16((dZ2 @ bf16(W2)^T) * [Z1 > 0]),  gW1 = X^T dZ1,  gb1 = column sums
    (dz w3^T uses bf16(w3));
  * Adam (Kingma and Ba, 2015) on the binary32 master parameters with bias
    correction: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr * m_hat /
    (sqrt(v_hat) + eps).

Here every step runs in float64 except the bfloat16 roundings, which are applied at
exactly the stated points; `exact=True` skips them (plain float64 network), which
is what the finite-difference pins check.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict

import numpy as np

K_IN = 288
HIDDEN = 256
PARAM_NAMES = ("W1", "b1", "W2", "b2", "w3", "b3")


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest even) through binary32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if nan.any():
        out = np.where(nan, f, out)
    return out.astype(np.float64)


@dataclass
class Params:
    W1: np.ndarray  # [K_IN, HIDDEN]
    b1: np.ndarray  # [HIDDEN]
    W2: np.ndarray  # [HIDDEN, HIDDEN]
    b2: np.ndarray  # [HIDDEN]
    w3: np.ndarray  # [HIDDEN]
    b3: np.ndarray  # [1]

    def as_dict(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in PARAM_NAMES}

    def copy(self) -> "Params":
        return Params(**{k: v.copy() for k, v in self.as_dict().items()})


def init_params(rng: np.random.Generator, in_dim: int) -> Params:
    """He-style init in binary32; rows of W1 at or past in_dim are zero."""
    W1 = np.zeros((K_IN, HIDDEN), np.float32)
    W1[:in_dim] = rng.standard_normal((in_dim, HIDDEN)) * np.sqrt(2.0 / in_dim)
    W2 = (rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN)).astype(np.float32)
    w3 = (rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN)).astype(np.float32)
    return Params(W1, np.zeros(HIDDEN, np.float32), W2, np.zeros(HIDDEN, np.float32), w3,
                  np.zeros(1, np.float32))


def pad_features(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f, np.float64)
    out = np.zeros((f.shape[0], K_IN))
    out[:, :f.shape[1]] = f
    return out


def forward(p: Params, f: np.ndarray, exact: bool = False):
    r = (lambda a: np.asarray(a, np.float64)) if exact else bf16
    X = r(pad_features(f))
    Z1 = X @ r(p.W1) + p.b1.astype(np.float64)
    A1 = r(np.maximum(Z1, 0.0))
    Z2 = A1 @ r(p.W2) + p.b2.astype(np.float64)
    A2 = r(np.maximum(Z2, 0.0))
    z = A2 @ r(p.w3) + float(p.b3[0])
    return z, (X, Z1, A1, Z2, A2)


def bce_with_logits(z: np.ndarray, y: np.ndarray) -> float:
    z = np.asarray(z, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_and_grads(p: Params, f: np.ndarray, y: np.ndarray, exact: bool = False):
    r = (lambda a: np.asarray(a, np.float64)) if exact else bf16
    y = np.asarray(y, np.float64)
    z, (X, Z1, A1, Z2, A2) = forward(p, f, exact)
    B = len(y)
    loss = bce_with_logits(z, y)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    g = {}
    g["w3"] = A2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dZ2 = r(np.outer(dz, r(p.w3)) * (Z2 > 0))
    g["W2"] = A1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = r((dZ2 @ r(p.W2).T) * (Z1 > 0))
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, g, z


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: Dict[str, np.ndarray] = field(default_factory=dict)
    v: Dict[str, np.ndarray] = field(default_factory=dict)

    def step(self, p: Params, g: Dict[str, np.ndarray]) -> Params:
        self.t += 1
        out = p.copy()
        for k in PARAM_NAMES:
            gk = np.asarray(g[k], np.float64)
            m = self.m.get(k, np.zeros_like(gk))
            v = self.v.get(k, np.zeros_like(gk))
            m = self.beta1 * m + (1 - self.beta1) * gk
            v = self.beta2 * v + (1 - self.beta2) * gk * gk
            self.m[k], self.v[k] = m, v
            mh = m / (1 - self.beta1 ** self.t)
            vh = v / (1 - self.beta2 ** self.t)
            setattr(out, k, (getattr(p, k).astype(np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps))
                    .astype(np.float32))
        return out


def obstacle_encoding(obs, n_slots: int = 40) -> np.ndarray:
    """Spheres as (centre, radius) in order, zero-padded to n_slots entries of d+1."""
    d = obs.d
    enc = np.zeros(n_slots * (d + 1))
    k = 0
    for o in range(len(obs.kind)):
        if k == n_slots:
            break
        if obs.kind[o] == 0:
            enc[k * (d + 1):k * (d + 1) + d] = obs.centre[o]
            enc[k * (d + 1) + d] = obs.size[o, 0]
            k += 1
    return enc


def features(points: np.ndarray, enc: np.ndarray) -> np.ndarray:
    pts = np.asarray(points, np.float64)
    return np.concatenate([pts, np.broadcast_to(enc, (len(pts), len(enc)))], axis=1)


def labels(g_root: np.ndarray, g_goal: np.ndarray, goal: int = 1, slack: float = 0.05) -> np.ndarray:
    """1 where a path through the vertex is within (1 + slack) of the best cost:
    g_root(v) + g_goal(v) <= (1 + slack) * g_root(goal) (in float64)."""
    best = float(g_root[goal])
    tot = np.asarray(g_root, np.float64) + np.asarray(g_goal, np.float64)
    return (np.isfinite(tot) & (tot <= (1.0 + slack) * best)).astype(np.float32)
