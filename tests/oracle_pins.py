"""Pins of the oracle to facts fixed outside it.

Each ``pin_*`` function takes a loaded oracle library (``oracle.load(path)``) and
raises AssertionError when the oracle disagrees with something the paper or the
mathematics fixes:

  * hand-worked examples (tests/golden/*.txt, each with its derivation);
  * FP64 shortest paths from SciPy's Dijkstra (pruning off: every reachable vertex;
    pruning on: the goal and every vertex the promising-set argument covers);
  * brute force over all simple paths on graphs of at most 9 vertices;
  * exact integer hop distances on unit-cost lattices;
  * the direct edge on complete obstacle-free graphs (triangle inequality);
  * the left fold of FP32 additions along each root path (closed form of Evaluate);
  * invariants: rooted acyclic tree, g(v) = g(parent) + c bitwise, pcost is a real
    edge, Bellman's inequality over the final Improve domain, monotone g across
    iterations, insertion-time local optimality, correctness from any initial
    policy (Sec. V), error returns.

The same functions run against copies of the oracle with planted mistakes
(test_oracle_mutants.py) to show that each plausible slip is caught.
"""
from __future__ import annotations

import glob
import itertools
import math
import os
from collections import deque

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
REL = 1e-5  # relative tolerance against FP64 shortest paths


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def load_fixture(path):
    fx = {"edges": [], "prune": 1, "h": None}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            if key == "edge":
                fx["edges"].append((int(rest[0]), int(rest[1]), float(rest[2])))
            elif key in ("n", "root", "goal", "prune"):
                fx[key] = int(rest[0])
            elif key in ("h", "insert_g", "expect_g"):
                fx[key] = np.array([float(x) for x in rest], np.float32)
            elif key in ("insert_parent", "expect_parent"):
                fx[key] = np.array([int(x) for x in rest], np.int32)
            elif key == "expect_stats":
                fx[key] = {k: int(v) for k, v in (kv.split("=") for kv in rest)}
            else:
                raise ValueError("unknown fixture key %r in %s" % (key, path))
    return fx


def fixtures():
    return sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))


def build_graph(lib, batches):
    G = O.Graph(lib)
    for b in batches:
        rc = G.insert_batch(b)
        assert rc == 0, "insert rc=%d" % rc
    return G


def sparse_of(G):
    ptr, nbr, cst = G.adjacency()
    n = G.n
    return sp.csr_matrix((cst.astype(np.float64), nbr, ptr), shape=(n, n))


def fp64_dist(G, root):
    # SciPy's Dijkstra keeps the smallest of parallel entries; explicit zeros
    # are dropped by csr -> use a tiny positive stand-in is not needed because
    # generator costs are > 0.
    return dijkstra(sparse_of(G), directed=False, indices=root)


def assert_close_fp64(g, d, mask, what):
    g64 = g.astype(np.float64)
    both = mask & np.isfinite(d)
    rel = np.abs(g64[both] - d[both]) / np.maximum(np.abs(d[both]), 1e-30)
    assert rel.size == 0 or rel.max() <= REL, "%s: max rel err %.3g" % (what, rel.max())


def fold_root_path(parent, pcost, root):
    """Closed form of Evaluate: g(v) is the left fold, in binary32, of the
    parent-edge costs along the root path of v (+inf if the chain misses root)."""
    n = len(parent)
    out = np.full(n, np.inf, np.float32)
    for v in range(n):
        path = []
        u = v
        seen = 0
        while u != root and u >= 0 and seen <= n:
            path.append(u)
            u = int(parent[u])
            seen += 1
        if u != root:
            continue
        acc = np.float32(0.0)
        for w in reversed(path):
            acc = np.float32(acc + pcost[w])
        out[v] = acc
    return out


def check_invariants(G, root, goal, h, prune):
    st = G.state()
    g, parent, pcost = st.g, st.parent, st.pcost
    n = G.n
    ptr, nbr, cst = G.adjacency()
    assert parent[root] == -1 and g[root] == 0.0
    # rooted, acyclic, consistent: the closed form reproduces g bit for bit
    fold = fold_root_path(parent, pcost, root)
    assert np.array_equal(fold.view(np.uint32), g.view(np.uint32)), "g is not the root-path fold"
    # each reachable vertex's parent edge exists with that exact cost
    for v in np.nonzero(np.isfinite(g))[0]:
        if v == root:
            continue
        p = parent[v]
        row = slice(ptr[v], ptr[v + 1])
        hits = (nbr[row] == p) & (cst[row].view(np.uint32) == np.float32(pcost[v]).view(np.uint32))
        assert hits.any(), "pcost of %d is not the cost of an edge to its parent" % v
    # Bellman at the fixed point over the final Improve domain
    thr = g[goal] if prune else np.float32(np.inf)
    hh = np.zeros(n, np.float32) if h is None else np.asarray(h, np.float32)
    f = (g + hh).astype(np.float32)
    P = f < thr
    D = P.copy()
    src = np.repeat(np.arange(n), np.diff(ptr))
    D[nbr[P[src]]] = True
    D[root] = False
    cand = (g[nbr] + cst).astype(np.float32)  # binary32 adds, elementwise
    bad = D[src] & (cand < g[src])
    assert not bad.any(), "Bellman inequality violated at %d vertices" % int(bad.sum())


# ----------------------------------------------------------------------------
# pins (cheap first: the mutant test stops at the first failure)
# ----------------------------------------------------------------------------

def pin_golden(lib):
    for path in fixtures():
        fx = load_fixture(path)
        G = build_graph(lib, [W.from_edges(fx["n"], fx["edges"])])
        st = G.state()
        name = os.path.basename(path)
        assert np.array_equal(st.g, fx["insert_g"]), "%s: insertion g %s" % (name, st.g)
        assert np.array_equal(st.parent, fx["insert_parent"]), "%s: insertion parent %s" % (name, st.parent)
        rc, stats = G.replan(fx["root"], fx["goal"], fx["h"], bool(fx["prune"]))
        assert rc == 0
        st = G.state()
        assert np.array_equal(st.g, fx["expect_g"]), "%s: g %s" % (name, st.g)
        assert np.array_equal(st.parent, fx["expect_parent"]), "%s: parent %s" % (name, st.parent)
        for k, v in fx["expect_stats"].items():
            assert stats[k] == v, "%s: %s=%d, expected %d" % (name, k, stats[k], v)


def pin_path_fold(lib):
    rng = np.random.default_rng(7)
    n = 200
    costs = rng.uniform(0.01, 1.0, n - 1).astype(np.float32)
    G = build_graph(lib, [W.path_graph(n, costs)])
    # insertion already gives the fold; Replan keeps it
    rc, stats = G.replan(0, n - 1, None, False)
    assert rc == 0 and stats["iterations"] == 1
    acc = np.float32(0.0)
    want = [acc]
    for c in costs:
        acc = np.float32(acc + c)
        want.append(acc)
    want = np.array(want, np.float32)
    assert np.array_equal(G.state().g.view(np.uint32), want.view(np.uint32))
    # the same path with reversed labels: every vertex but 0 starts as an orphan
    # except along the chain, and Replan must rebuild the fold from the root 0.
    rev = n - 1 - np.arange(n)  # new label of old vertex i
    edges = [(int(rev[i]), int(rev[i + 1]), float(costs[i])) for i in range(n - 1)]
    G2 = build_graph(lib, [W.from_edges(n, edges)])
    root = int(rev[0])
    rc, _ = G2.replan(root, int(rev[n - 1]), None, False)
    assert rc == 0
    g2 = G2.state().g
    assert np.array_equal(g2[rev].view(np.uint32), want.view(np.uint32))


def pin_bruteforce_small(lib):
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(2, 10))
        edges = []
        for a in range(n):
            for b in range(a + 1, n):
                if rng.random() < 0.45:
                    edges.append((a, b, float(np.float32(rng.uniform(0.1, 2.0)))))
        adj = {v: [] for v in range(n)}
        for a, b, c in edges:
            adj[a].append((b, c))
            adj[b].append((a, c))

        def best_from(root):
            best = [math.inf] * n
            best[root] = 0.0

            def dfs(u, acc, seen):
                for w, c in adj[u]:
                    if w in seen:
                        continue
                    t = acc + c
                    if t < best[w]:
                        best[w] = t
                    dfs(w, t, seen | {w})
            dfs(root, 0.0, {root})
            return np.array(best)

        dist = [best_from(v) for v in range(n)]
        for root in range(n):
            d = dist[root]
            for goal in range(n):
                if goal == root:
                    continue
                dg = dist[goal]
                # admissible heuristic: half the true cost-to-go (0 where unreachable)
                h_half = np.where(np.isfinite(dg), 0.5 * dg, 0.0).astype(np.float32)
                for h in (None, h_half):
                    for prune in (False, True):
                        G2 = build_graph(lib, [W.from_edges(n, edges)])
                        rc, _ = G2.replan(root, goal, h, prune)
                        assert rc == 0
                        g = G2.state().g
                        if not prune:
                            assert (np.isfinite(g) == np.isfinite(d)).all(), "reachable set differs"
                            assert_close_fp64(g, d, np.ones(n, bool), "bruteforce n=%d" % n)
                        elif np.isfinite(d[goal]):
                            assert_close_fp64(g, d, np.arange(n) == goal, "bruteforce goal")
                        else:
                            assert not np.isfinite(g[goal])


def pin_lattice(lib):
    rng = np.random.default_rng(3)
    side = 14
    keep = rng.random((side, side)) > 0.15
    keep[0, 0] = keep[side - 1, side - 1] = True
    cells = [(i, j) for i in range(side) for j in range(side) if keep[i, j]]
    perm = rng.permutation(len(cells))
    # the root keeps label 0 so that insertion sees it first; the rest are shuffled
    start = cells.index((0, 0))
    order = [start] + [k for k in perm if k != start]
    label = {cells[k]: i for i, k in enumerate(order)}
    edges = []
    for (i, j) in cells:
        for (a, b) in ((i + 1, j), (i, j + 1)):
            if (a, b) in label:
                edges.append((label[(i, j)], label[(a, b)], 1.0))
    n = len(cells)
    G = build_graph(lib, [W.from_edges(n, edges)])
    goal = label[(side - 1, side - 1)]
    rc, _ = G.replan(0, goal, None, False)
    assert rc == 0
    # plain BFS hop distances
    adj = [[] for _ in range(n)]
    for a, b, _ in edges:
        adj[a].append(b)
        adj[b].append(a)
    hop = np.full(n, np.inf)
    hop[0] = 0
    q = deque([0])
    while q:
        u = q.popleft()
        for w in adj[u]:
            if hop[w] == np.inf:
                hop[w] = hop[u] + 1
                q.append(w)
    assert np.array_equal(G.state().g, hop.astype(np.float32)), "lattice hop distances differ"


def pin_complete_graph(lib):
    rng = np.random.default_rng(5)
    n = 48
    pts = rng.random((n, 2))
    edges = []
    c = np.zeros((n, n), np.float32)
    for a in range(n):
        for b in range(a + 1, n):
            c[a, b] = c[b, a] = np.float32(np.sqrt(((pts[a] - pts[b]) ** 2).sum()))
            edges.append((a, b, float(c[a, b])))
    G = build_graph(lib, [W.from_edges(n, edges)])
    rc, _ = G.replan(0, 1, None, False)
    assert rc == 0
    st = G.state()
    # a two-hop route can only beat the direct edge through FP32 rounding
    for v in range(1, n):
        two = min(np.float32(c[0, u] + c[u, v]) for u in range(1, n) if u != v)
        if two > c[0, v]:
            assert st.g[v] == c[0, v] and st.parent[v] == 0, "vertex %d" % v
        else:
            assert st.g[v] <= c[0, v]


def pin_dijkstra(lib):
    wl = W.plain_2d(samples=600, seed=0)
    for root, goal in ((0, 1), (1, 0), (5, 17)):
        G = build_graph(lib, wl.batches)
        rc, _ = G.replan(root, goal, None, False)
        assert rc == 0
        d = fp64_dist(G, root)
        g = G.state().g
        assert (np.isfinite(g) == np.isfinite(d)).all(), "reachable set differs"
        assert_close_fp64(g, d, np.ones(G.n, bool), "2D root %d" % root)
    wl6 = W.batched_6d(batches=4, batch=300, seed=100)
    G = O.Graph(lib)
    for b in wl6.batches:
        assert G.insert_batch(b) == 0
        rc, _ = G.replan(0, 1, None, False)
        assert rc == 0
        d = fp64_dist(G, 0)
        g = G.state().g
        assert (np.isfinite(g) == np.isfinite(d)).all()
        assert_close_fp64(g, d, np.ones(G.n, bool), "6D n=%d" % G.n)


def pin_pruned_exactness(lib):
    """With an admissible, consistent h and pruning on: g(goal) is optimal, and so
    is g(v) for every v with d(v) + h(v) < d(goal) (margin 1e-4 for rounding)."""
    for wl in (W.plain_2d(samples=800, seed=0), W.batched_6d(batches=3, batch=400, seed=100)):
        G = O.Graph(lib)
        for b in wl.batches:
            assert G.insert_batch(b) == 0
            h = wl.heuristic(G.n)
            rc, _ = G.replan(0, 1, h, True)
            assert rc == 0
            d = fp64_dist(G, 0)
            g = G.state().g
            if np.isfinite(d[1]):
                mask = (np.arange(G.n) == 1) | (d + h.astype(np.float64) < d[1] * (1 - 1e-4))
                assert_close_fp64(g, d, mask, "%s pruned" % wl.name)
            check_invariants(G, 0, 1, h, True)


def pin_invariants(lib):
    wl = W.plain_2d(samples=1000, seed=0)
    for prune in (True, False):
        G = build_graph(lib, wl.batches)
        h = wl.heuristic()
        rc, _ = G.replan(0, 1, h, prune)
        assert rc == 0
        check_invariants(G, 0, 1, h, prune)


def pin_insertion_local(lib):
    """Extend's local relaxation: each new vertex's (g, parent) is the smallest
    (g(u) + c, u) over its lower-index neighbours, or an orphan if none is finite."""
    wl = W.batched_6d(batches=3, batch=300, seed=100)
    G = O.Graph(lib)
    for b in wl.batches:
        assert G.insert_batch(b) == 0
        st = G.state()
        for i in range(b.n_new):
            v = b.n_old + i
            if v == 0:
                assert st.g[0] == 0 and st.parent[0] == -1
                continue
            cols = b.col[b.row_ptr[i]:b.row_ptr[i + 1]]
            cs = b.cost[b.row_ptr[i]:b.row_ptr[i + 1]]
            cands = sorted((float(np.float32(st.g[u] + c)), int(u)) for u, c in zip(cols, cs))
            finite = [x for x in cands if math.isfinite(x[0])]
            if not finite:
                assert st.parent[v] == -1 and np.isinf(st.g[v])
            else:
                assert (float(st.g[v]), int(st.parent[v])) == finite[0], "vertex %d" % v
        rc, _ = G.replan(0, 1, wl.heuristic(G.n), True)
        assert rc == 0


def pin_any_initial_policy(lib):
    """Sec. V: Replan over the whole graph recovers the optimum from any initial
    policy: one batch, many batches, and an all-orphan start agree with FP64."""
    wl = W.plain_2d(samples=700, seed=0)
    whole = build_graph(lib, wl.batches)
    d = fp64_dist(whole, 0)
    pts = wl.points
    # the same graph split into 7 batches
    edges = []
    b = wl.batches[0]
    for i in range(b.n_new):
        for j in range(b.row_ptr[i], b.row_ptr[i + 1]):
            edges.append((i, int(b.col[j]), float(b.cost[j])))
    cuts = [0, 2, 100, 200, 300, 400, 500, len(pts)]
    G = O.Graph(lib)
    for a, z in zip(cuts[:-1], cuts[1:]):
        assert G.insert_batch(W.from_edges(z, [e for e in edges if a <= max(e[0], e[1]) < z], n_old=a)) == 0
    rc, _ = G.replan(0, 1, None, False)
    assert rc == 0
    assert (np.isfinite(G.state().g) == np.isfinite(d)).all()
    assert_close_fp64(G.state().g, d, np.ones(G.n, bool), "7 batches")
    # all orphans
    G3 = build_graph(lib, wl.batches)
    n = G3.n
    assert G3.set_state(np.full(n, np.inf, np.float32), np.full(n, -1, np.int32), np.zeros(n, np.float32)) == 0
    rc, _ = G3.replan(0, 1, None, False)
    assert rc == 0
    assert_close_fp64(G3.state().g, d, np.ones(n, bool), "all orphans")


def pin_monotone(lib):
    """g never increases from one policy-iteration step to the next, and the
    iteration cap returns ENOTCONVERGED with a consistent state."""
    wl = W.plain_2d(samples=600, seed=0)
    base = build_graph(lib, wl.batches)
    st0 = base.state()
    h = wl.heuristic()
    rc, full = base.replan(0, 1, h, True)
    assert rc == 0
    total = full["iterations"]
    prev = None
    for k in range(1, total + 1):
        G = build_graph(lib, wl.batches)
        assert G.set_state(st0.g, st0.parent, st0.pcost) == 0
        rc, stats = G.replan(0, 1, h, True, max_iters=k)
        if k < total:
            assert rc == O.ENOTCONVERGED and stats["iterations"] == k, (k, rc, stats)
        else:
            assert rc == 0
        g = G.state().g
        fold = fold_root_path(G.state().parent, G.state().pcost, 0)
        assert np.array_equal(fold.view(np.uint32), g.view(np.uint32))
        if prev is not None:
            assert (g <= prev).all(), "g increased at step %d" % k
        prev = g


def pin_errors(lib):
    G = O.Graph(lib)
    assert G.insert(np.array([0, 1], np.int64), np.array([0], np.int32), np.array([1.0], np.float32)) == O.EINVAL
    assert G.n == 0
    assert G.insert(np.array([0, 0, 1], np.int64), np.array([0], np.int32), np.array([np.nan], np.float32)) == O.EINVAL
    assert G.insert(np.array([0, 0, 1], np.int64), np.array([0], np.int32), np.array([-1.0], np.float32)) == O.EINVAL
    assert G.insert(np.array([0, 0, 1], np.int64), np.array([0], np.int32), np.array([1.0], np.float32)) == 0
    assert G.replan(2, 0)[0] == O.EINVAL
    assert G.replan(0, 1, np.array([0.0, np.nan], np.float32))[0] == O.EINVAL
    assert G.replan(0, 1, np.array([0.0, -1.0], np.float32))[0] == O.EINVAL


def lookahead_example():
    """A five-vertex graph worked by hand for the narrowed Improve domain.

    Edges 0-2 (1), 2-1 (1), 0-3 (0.5), 3-1 (3), 2-4 (0.5); root 0, goal 1;
    h = (1, 0, 0.5, 1.2, 1); starting policy 2<-0, 1<-2, 3<-1, 4<-2, so
    g = (0, 2, 1, 5, 1.5) and G = g(1) = 2, f = g + h = (1, 2, 1.5, 6.2, 2.5).
    Iteration 1: P = {0, 2}.  Full domain: P and its neighbours minus the root
    = {1, 2, 3, 4} (degrees 2 + 3 + 2 + 1 = 8 entries).  Narrowed: from 0 the
    offers are 1 + 0.5 = 1.5 to 2 and 0.5 + 1.2 = 1.7 to 3 (both < 2); from 2 they
    are 2 + 1 = 3 to 0, 2 + 0 = 2 to 1, 1.5 + 1 = 2.5 to 4 (none < 2): D = {2, 3}
    (5 entries).  Improve moves 3 under 0 (0.5 < 5).  Iteration 2: g(3) = 0.5,
    P = {0, 2, 3}; the full domain is again {1, 2, 3, 4}; from 3 the offers are
    1 + 1 = 2 to 0 and 3.5 to 1, so the narrowed domain stays {2, 3}; nothing
    changes.  Totals (iterations, sum_P, sum_D, edges, changed): full mode
    (2, 5, 8, 16, 1), narrowed (2, 5, 4, 10, 1); final g = (0, 2, 1, 0.5, 1.5).
    The promising rows walked to build the domain are the same in both modes:
    deg 0 + deg 2 = 5 entries, then deg 0 + deg 2 + deg 3 = 7, so mark_edges = 12."""
    edges = [(0, 2, 1.0), (2, 1, 1.0), (0, 3, 0.5), (3, 1, 3.0), (2, 4, 0.5)]
    h = np.array([1.0, 0.0, 0.5, 1.2, 1.0], np.float32)
    parent = np.array([-1, 2, 0, 1, 2], np.int32)
    pcost = np.array([0.0, 1.0, 1.0, 3.0, 0.5], np.float32)
    return edges, h, parent, pcost


def pin_lookahead_worked_example(lib):
    edges, h, parent, pcost = lookahead_example()
    want = {False: (2, 5, 8, 16, 1), True: (2, 5, 4, 10, 1)}
    for look in (False, True):
        G = build_graph(lib, [W.from_edges(5, edges)])
        assert G.set_state(np.zeros(5, np.float32), parent, pcost) == 0
        rc, st = G.replan(0, 1, h, True, lookahead=look)
        assert rc == 0
        got = (st["iterations"], st["sum_P"], st["sum_D"], st["edges_examined"], st["changed_total"])
        assert got == want[look], (look, got)
        assert st["mark_edges"] == 12, (look, st["mark_edges"])
        fin = G.state()
        assert np.array_equal(fin.g, np.array([0, 2, 1, 0.5, 1.5], np.float32))
        assert np.array_equal(fin.parent, np.array([-1, 2, 0, 0, 2], np.int32))


def pin_lookahead_properties(lib):
    """Narrowed domain: without pruning it is the full domain (G = +inf passes every
    finite offer), so results and counters coincide; with pruning and a consistent h
    the exactness argument still holds (the next vertex of an optimal path is offered
    its optimal value by a promising predecessor), so g(goal) and every vertex with
    d(v) + h(v) < d(goal) are optimal; it never takes more entries than the full
    domain in the first iteration; and the fixed point satisfies the invariants."""
    for wl in (W.plain_2d(samples=800, seed=0), W.batched_6d(batches=3, batch=400, seed=100)):
        G = build_graph(lib, wl.batches)
        H = build_graph(lib, wl.batches)
        h = wl.heuristic(G.n)
        rc1, s1 = G.replan(0, 1, h, False, lookahead=True)
        rc2, s2 = H.replan(0, 1, h, False, lookahead=False)
        assert rc1 == rc2 == 0 and s1 == s2, (s1, s2)
        a, b = G.state(), H.state()
        assert np.array_equal(a.g.view(np.uint32), b.g.view(np.uint32)) and np.array_equal(a.parent, b.parent)
        # first iteration from the same policy: the narrowed domain is a subset
        G = build_graph(lib, wl.batches)
        H = build_graph(lib, wl.batches)
        _, f1 = G.replan(0, 1, h, True, max_iters=1, lookahead=True)
        _, f2 = H.replan(0, 1, h, True, max_iters=1, lookahead=False)
        assert f1["sum_P"] == f2["sum_P"] and f1["sum_D"] <= f2["sum_D"]
        assert f1["edges_examined"] <= f2["edges_examined"]
        G = build_graph(lib, wl.batches)
        rc, st = G.replan(0, 1, h, True, lookahead=True)
        assert rc == 0
        d = fp64_dist(G, 0)
        g = G.state().g
        if np.isfinite(d[1]):
            mask = (np.arange(G.n) == 1) | (d + h.astype(np.float64) < d[1] * (1 - 1e-4))
            assert_close_fp64(g, d, mask, "%s narrowed" % wl.name)
        fold = fold_root_path(G.state().parent, G.state().pcost, 0)
        assert np.array_equal(fold.view(np.uint32), g.view(np.uint32))


def truncated_example():
    """A six-vertex graph worked by hand for the truncated Evaluate.

    Edges 0-1 (4), 0-2 (3), 0-5 (1), 5-2 (1), 2-3 (3), 3-4 (1); root 0, goal 1,
    h = 0, pruning on; starting policy 1<-0, 2<-0, 3<-2, 4<-3, 5<-0 with its
    consistent g = (0, 4, 3, 6, 7, 1).
    First Evaluate: G0 = g(1) = 4.  From the root: g(1) = 4 (not < 4, not queued),
    g(2) = 3 and g(5) = 1 (queued, B = {2, 5}); from 2: g(3) = 6 (not queued); 4 is
    not reached and keeps 7.
    Iteration 1: P = {2, 5}; D = {2, 5} and their neighbours minus the root =
    {2, 3, 5} (degrees 3 + 2 + 2 = 7 entries).  Improve: 2 has 0+3, 1+1 = 2, 6+3 -> it
    moves under 5 (2 < 3); 3 has 3+3 = 6 and 7+1 = 8 (6 is not below 6); 5 keeps 0.
    Evaluate: G0 = 4; g(1) = 4 (not queued), g(5) = 1 (queued), then g(2) = 2
    (queued), then g(3) = 2 + 3 = 5 (not queued); 4 is not reached: g(4) stays 7
    although its path now costs 6.
    Iteration 2: P = {2, 5}, D = {2, 3, 5} again; nothing switches (2 has 2, 3 has
    5 and 7 + 1, 5 has 1).  Totals (iterations, sum_P, sum_D, edges, changed) =
    (2, 4, 6, 14, 1); final g = (0, 4, 2, 5, 7, 1), parents (-1, 0, 5, 2, 3, 0).
    The full mode from the same policy puts the root in P (D = {1, 2, 3, 5}), ends
    with g(4) = 6 and counts (2, 6, 8, 16, 1)."""
    edges = [(0, 1, 4.0), (0, 2, 3.0), (0, 5, 1.0), (5, 2, 1.0), (2, 3, 3.0), (3, 4, 1.0)]
    parent = np.array([-1, 0, 0, 2, 3, 0], np.int32)
    pcost = np.array([0.0, 4.0, 3.0, 3.0, 1.0, 1.0], np.float32)
    g = np.array([0.0, 4.0, 3.0, 6.0, 7.0, 1.0], np.float32)
    return edges, g, parent, pcost


def pin_truncated_worked_example(lib):
    edges, g0, parent, pcost = truncated_example()
    want = {True: ((2, 4, 6, 14, 1), [0, 4, 2, 5, 7, 1]), False: ((2, 6, 8, 16, 1), [0, 4, 2, 5, 6, 1])}
    for trunc in (True, False):
        G = build_graph(lib, [W.from_edges(6, edges)])
        assert G.set_state(g0, parent, pcost) == 0
        rc, st = G.replan(0, 1, np.zeros(6, np.float32), True, truncated=trunc)
        assert rc == 0
        got = (st["iterations"], st["sum_P"], st["sum_D"], st["edges_examined"], st["changed_total"])
        assert got == want[trunc][0], (trunc, got)
        fin = G.state()
        assert np.array_equal(fin.g, np.array(want[trunc][1], np.float32)), (trunc, fin.g)
        assert np.array_equal(fin.parent, np.array([-1, 0, 5, 2, 3, 0], np.int32))
    G = build_graph(lib, [W.from_edges(6, edges)])
    assert G.replan(0, 1, None, True, truncated=True, lookahead=True)[0] == O.EINVAL


def pin_truncated_properties(lib):
    """Truncated Evaluate: without pruning (G0 = +inf) every vertex the root reaches
    is visited and queued, so from the insertion-time state -- where every neighbour
    of vertex 0 is attached to the tree and every unattached vertex holds +inf -- B is
    the full mode's P minus the root, N(root) lies in B, and the two modes give the
    same counters and bits.  With pruning, the first iteration's B lies inside the full
    mode's P minus the root (the visited vertices get the same values from a
    consistent start, and each of them passed the same test), so its domain is no
    larger; g(goal) is still the cost of a path, so never below the FP64 shortest
    distance."""
    for wl in (W.plain_2d(samples=800, seed=0), W.batched_6d(batches=3, batch=400, seed=100)):
        G = build_graph(lib, wl.batches)
        H = build_graph(lib, wl.batches)
        h = wl.heuristic(G.n)
        rc1, s1 = G.replan(0, 1, h, False, truncated=True)
        rc2, s2 = H.replan(0, 1, h, False)
        assert rc1 == rc2 == 0
        # the root is in every full-mode P (and its row is walked for the domain)
        deg0 = int(np.diff(H.adjacency()[0])[0])
        s2 = dict(s2, sum_P=s2["sum_P"] - s2["iterations"], mark_edges=s2["mark_edges"] - s2["iterations"] * deg0)
        assert s1 == s2, (wl.name, s1, s2)
        a, b = G.state(), H.state()
        assert np.array_equal(a.g.view(np.uint32), b.g.view(np.uint32)) and np.array_equal(a.parent, b.parent)
        G = build_graph(lib, wl.batches)
        H = build_graph(lib, wl.batches)
        _, f1 = G.replan(0, 1, h, True, max_iters=1, truncated=True)
        _, f2 = H.replan(0, 1, h, True, max_iters=1)
        assert f1["sum_P"] < f2["sum_P"] and f1["sum_D"] <= f2["sum_D"], (f1, f2)  # the root is in P
        assert f1["edges_examined"] <= f2["edges_examined"]
        G = build_graph(lib, wl.batches)
        rc, st = G.replan(0, 1, h, True, truncated=True)
        assert rc == 0
        d = fp64_dist(G, 0)
        g1 = float(G.state().g[1])
        assert np.isfinite(d[1]) == np.isfinite(g1)
        if np.isfinite(g1):
            assert g1 >= d[1] * (1 - 1e-4), (wl.name, g1, d[1])


def pin_row_order(lib):
    """Metamorphic: shuffling the entries inside every input row changes neither the
    insertion-time policy nor the Replan (both take lexicographic minima, so the order
    in which candidates are met cannot matter), including on a lattice full of ties."""
    import dataclasses
    rng = np.random.default_rng(5)
    for wl in (W.plain_2d(samples=1500, seed=12), W.batched_6d(batches=2, batch=300, seed=110)):
        shuffled = []
        for b in wl.batches:
            col, cost = b.col.copy(), b.cost.copy()
            for v in range(b.n_new):
                a, e = int(b.row_ptr[v]), int(b.row_ptr[v + 1])
                perm = a + rng.permutation(e - a)
                col[a:e], cost[a:e] = b.col[perm], b.cost[perm]
            shuffled.append(dataclasses.replace(b, col=col, cost=cost))
        outs = []
        for batches in (wl.batches, shuffled):
            G = build_graph(lib, batches)
            ins = G.state()
            rc, st = G.replan(0, 1, wl.heuristic(G.n), True)
            assert rc == 0
            fin = G.state()
            outs.append((ins.g.view(np.uint32).copy(), ins.parent.copy(), fin.g.view(np.uint32).copy(),
                         fin.parent.copy(), st))
        for x, y in zip(outs[0], outs[1]):
            assert (x == y) if isinstance(x, dict) else np.array_equal(x, y), wl.name


def pin_mark_edges(lib):
    """mark_edges by brute force: iteration k's promising set recomputed from the
    state after k - 1 iterations (a Replan capped there, or the first Evaluate), in
    binary32, and its rows' degrees summed from the adjacency."""
    wl = W.plain_2d(samples=300, seed=3)
    for prune in (True, False):
        G = build_graph(lib, wl.batches)
        h = wl.heuristic()
        rc, st = G.replan(0, 1, h, prune)
        assert rc == 0
        deg = np.diff(G.adjacency()[0])
        total = 0
        for k in range(1, st["iterations"] + 1):
            H = build_graph(lib, wl.batches)
            if k == 1:
                assert H.evaluate(0) >= 0  # the tree levels walked
            else:
                rc_k, _ = H.replan(0, 1, h, prune, max_iters=k - 1)
                assert rc_k == O.ENOTCONVERGED
            g = H.state().g
            thr = g[1] if prune else np.float32(np.inf)
            total += int(deg[(g + h) < thr].sum())
        assert st["mark_edges"] == total, (prune, st["mark_edges"], total)


PINS = [pin_golden, pin_path_fold, pin_errors, pin_lattice, pin_complete_graph, pin_insertion_local,
        pin_monotone, pin_invariants, pin_dijkstra, pin_pruned_exactness, pin_any_initial_policy,
        pin_bruteforce_small, pin_lookahead_worked_example, pin_lookahead_properties,
        pin_truncated_worked_example, pin_truncated_properties, pin_row_order, pin_mark_edges]
