"""Seeded random cases against the oracle: batches of mixed problems (tiny hand-made
graphs next to RRGs of 2D-8D, so problems share tiles), random roots and goals, a
second Replan with new roots on the same handle, and single graphs grown in several
batches on both sides of the size from which the mark's listed rows take half a grid.  g bit for bit,
parents and every counter exactly, as in the other parity tests."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_batch import Problem, build, check_problem, concat_rows, full_h, oracle_run
from test_gpu_parity import STAT_KEYS, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


@pytest.fixture(autouse=True)
def device_path(monkeypatch):
    monkeypatch.setenv("PIRRT_HOST_MAX", "0")


def random_problem(rng):
    if rng.random() < 0.25:
        n = int(rng.integers(1, 6))
        edges = [(a, b, float(rng.random())) for a in range(n) for b in range(a) if rng.random() < 0.6]
        b = W.from_edges(n, edges)
        rows, h, name = (b.row_ptr, b.col, b.cost), None, "tiny-%d" % n
    else:
        wl = W.multi_problem(int(rng.integers(0, 10**6)), base_seed=int(rng.integers(0, 10**6)), n_min=200,
                             n_max=int(rng.choice([3000, 9000, 20000])))
        rows, h, name = concat_rows(wl.batches), wl.heuristic(wl.n), wl.name
    n = len(rows[0]) - 1
    root = 0 if rng.random() < 0.7 else int(rng.integers(0, n))
    goal = 1 % n if rng.random() < 0.7 else int(rng.integers(0, n))
    return Problem(name, rows, root, goal, h)


@pytest.mark.parametrize("seed", range(12))
def test_random_batch(P, seed):
    rng = np.random.default_rng(5000 + seed)
    probs = [random_problem(rng) for _ in range(int(rng.integers(2, 14)))]
    prune = bool(rng.random() < 0.8)
    for pr in probs:
        pr.prune = prune
    B = build(P, probs)
    off = B.offsets
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs), prune)
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("seed %d" % seed, g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (seed, pr.name, k)
    # a second Replan on the same handle from new roots (the captured loop replayed)
    roots2 = [int(rng.integers(0, p.n)) for p in probs]
    g, parent, stats = B.replan(roots2, [p.goal for p in probs], full_h(probs), prune)
    for i, pr in enumerate(probs):
        R = O.Graph()
        rp, col, cst = pr.rows
        assert R.insert_batch(W.Batch(0, pr.n, rp, col, cst, 0.0)) == 0
        R.replan(pr.root, pr.goal, pr.h, prune)
        rc, st = R.replan(roots2[i], pr.goal, pr.h, prune)
        fin = R.state()
        check_problem("seed %d, second Replan" % seed, g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (seed, pr.name, k)


@pytest.mark.parametrize("seed,d,n_total,k", [(1, 2, 40000, 3), (2, 3, 150000, 2), (3, 6, 300000, 1)])
def test_random_single_graph(P, seed, d, n_total, k):
    """300k vertices are above the size from which the listed rows take half a grid."""
    rng = np.random.default_rng(6000 + seed)
    obs = W.make_obstacles(d, int(rng.integers(5, 30)), "mixed", int(rng.integers(0, 10**6)))
    sizes = [n_total // k] * k
    wl = W.grow("random-%dd" % d, d, obs, int(rng.integers(0, 10**6)), sizes)
    plan = {i: (0 if rng.random() < 0.6 else int(rng.integers(0, sum(sizes[:i + 1]) + 2)), 1) for i in range(k)}
    run_both(P, wl.batches, plan, h_of=lambda n: wl.heuristic(n), prune=bool(rng.random() < 0.85),
             check_insert=False)
