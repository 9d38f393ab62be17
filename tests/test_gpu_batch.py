"""Batched Replan (pirrt_batch_* through the C ABI): every problem of a batch must
end exactly where the oracle ends on a graph holding that problem alone -- g bit for
bit, parents, and the per-problem statistics."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle_pins import fixtures, load_fixture

pytestmark = pytest.mark.gpu

STAT_KEYS = ("iterations", "edges_examined", "sum_P", "sum_D", "changed_total", "mark_edges")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


def gpu_batch(P, **kw):
    import torch
    return P.Batch(stream=torch.cuda.current_stream().cuda_stream, **kw)


def concat_rows(batches):
    """One problem from several insertion batches (forward rows, ids unchanged)."""
    ptr = [np.zeros(1, np.int64)]
    cols, costs, base = [], [], 0
    for b in batches:
        ptr.append(b.row_ptr[1:] + base)
        cols.append(b.col)
        costs.append(b.cost)
        base += int(b.row_ptr[-1])
    return (np.concatenate(ptr), np.concatenate(cols).astype(np.int32), np.concatenate(costs).astype(np.float32))


class Problem:
    def __init__(self, name, rows, root, goal, h, prune=True):
        self.name, self.rows, self.root, self.goal, self.h, self.prune = name, rows, root, goal, h, prune
        self.n = len(rows[0]) - 1


def problem_set():
    """A mixed set: RRGs of several dimensions and sizes, a lattice with exact ties,
    a golden fixture, a one-vertex problem and a disconnected one."""
    out = []
    for i in range(5):
        wl = W.multi_problem(i, n_min=800, n_max=12_000)
        out.append(Problem(wl.name, concat_rows(wl.batches), 0, 1, wl.heuristic(wl.n)))
    wl = W.batched_6d(batches=4, batch=600, seed=105)
    out.append(Problem(wl.name, concat_rows(wl.batches), 0, 1, wl.heuristic(wl.n)))
    fx = next(f for f in map(load_fixture, fixtures()) if f["prune"] == 1)
    b = W.from_edges(fx["n"], fx["edges"])
    out.append(Problem("fixture", (b.row_ptr, b.col, b.cost), fx["root"], fx["goal"],
                       None if fx["h"] is None else np.asarray(fx["h"], np.float32)))
    out.append(Problem("one-vertex", (np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)),
                       0, 0, np.zeros(1, np.float32)))
    b = W.from_edges(6, [(0, 1, 1.0), (1, 2, 0.5), (3, 4, 2.0), (4, 5, 1.0)])
    out.append(Problem("two-components", (b.row_ptr, b.col, b.cost), 0, 2, np.zeros(6, np.float32)))
    out.append(lattice(40, seed=7))
    return out


def lattice(side, seed):
    """A side x side grid with unit costs (many exactly tied paths), vertex ids
    shuffled, root and goal at opposite corners."""
    rng = np.random.default_rng(seed)
    n = side * side
    perm = rng.permutation(n)
    edges = []
    for r in range(side):
        for c in range(side):
            v = r * side + c
            if c + 1 < side:
                edges.append((int(perm[v]), int(perm[v + 1]), 1.0))
            if r + 1 < side:
                edges.append((int(perm[v]), int(perm[v + side]), 1.0))
    b = W.from_edges(n, edges)
    return Problem("lattice-%d" % side, (b.row_ptr, b.col, b.cost), int(perm[0]), int(perm[n - 1]),
                   np.zeros(n, np.float32))


def oracle_run(pr, root=None, goal=None, prune=None):
    R = O.Graph()
    rp, col, cst = pr.rows
    assert R.insert_batch(W.Batch(0, pr.n, rp, col, cst, 0.0)) == 0
    ins = R.state()
    rc, st = R.replan(pr.root if root is None else root, pr.goal if goal is None else goal, pr.h,
                      pr.prune if prune is None else prune)
    return ins, rc, st, R.state()


def full_h(probs):
    return np.concatenate([np.zeros(p.n, np.float32) if p.h is None else np.asarray(p.h, np.float32)
                           for p in probs])


def check_problem(tag, g, parent, off, pr, want_g, want_parent):
    g = np.asarray(g)[off:off + pr.n]
    parent = np.asarray(parent)[off:off + pr.n]
    bad_g = np.nonzero(g.view(np.uint32) != want_g.view(np.uint32))[0]
    bad_p = np.nonzero(parent != want_parent)[0]
    assert bad_g.size == 0, "%s %s: %d g mismatches, first %s" % (tag, pr.name, bad_g.size, bad_g[:5])
    assert bad_p.size == 0, "%s %s: %d parent mismatches, first %s: %s vs %s" % (
        tag, pr.name, bad_p.size, bad_p[:5], parent[bad_p[:5]], want_parent[bad_p[:5]])


def build(P, probs, **kw):
    B = gpu_batch(P, **kw)
    for i, pr in enumerate(probs):
        assert B.add_problem(*pr.rows) == i
    assert B.num_problems == len(probs)
    assert B.n == sum(p.n for p in probs)
    return B


def test_batch_matches_single_problems(P):
    probs = problem_set()
    B = build(P, probs)
    off = B.offsets
    assert off[-1] == B.n
    # insertion-time policy of every problem
    g0, p0, _ = B.get_policy()
    want = [oracle_run(pr) for pr in probs]
    for i, pr in enumerate(probs):
        check_problem("insert", g0, p0, off[i], pr, want[i][0].g, want[i][0].parent)
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    for i, pr in enumerate(probs):
        ins, rc, st, fin = want[i]
        assert rc == 0 and stats[i]["rc"] == 0
        check_problem("replan", g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k, stats[i][k], st[k])


def test_batch_second_replan_and_repeat(P):
    """A second Replan with other roots (old root marks must go), then the same
    Replan repeated from a snapshot: every repeat identical (the captured loop
    bodies are replayed)."""
    probs = problem_set()[:4]
    B = build(P, probs)
    off = B.offsets
    B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    B.snapshot_save()
    roots = [p.goal for p in probs]
    goals = [p.root for p in probs]
    results = []
    for rep in range(3):
        B.snapshot_restore()
        g, parent, stats = B.replan(roots, goals, None, prune=False)
        results.append((g.copy(), parent.copy(), [s["iterations"] for s in stats]))
    for i, pr in enumerate(probs):
        R = O.Graph()
        assert R.insert_batch(W.Batch(0, pr.n, *pr.rows, 0.0)) == 0
        assert R.replan(pr.root, pr.goal, pr.h, True)[0] == 0
        rc, st = R.replan(pr.goal, pr.root, None, False)
        assert rc == 0
        fin = R.state()
        for g, parent, its in results:
            check_problem("goal-rooted", g, parent, off[i], pr, fin.g, fin.parent)
            assert its[i] == st["iterations"]


def test_batch_add_after_replan(P):
    probs = problem_set()
    B = build(P, probs[:3])
    B.replan([p.root for p in probs[:3]], [p.goal for p in probs[:3]], full_h(probs[:3]))
    for pr in probs[3:6]:
        B.add_problem(*pr.rows)
    sel = probs[:6]
    off = B.offsets
    g, parent, stats = B.replan([p.root for p in sel], [p.goal for p in sel], full_h(sel))
    for i, pr in enumerate(sel):
        R = O.Graph()
        assert R.insert_batch(W.Batch(0, pr.n, *pr.rows, 0.0)) == 0
        if i < 3:  # replanned twice, as on the device
            assert R.replan(pr.root, pr.goal, pr.h, True)[0] == 0
        rc, st = R.replan(pr.root, pr.goal, pr.h, True)
        assert rc == 0
        fin = R.state()
        check_problem("after add", g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k)


def test_batch_device_buffers(P):
    import torch
    probs = problem_set()[:5]
    B = gpu_batch(P)
    for pr in probs:
        B.add_problem(*(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in pr.rows))
    off = B.offsets
    h = torch.from_numpy(full_h(probs)).cuda()
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], h)
    assert g.is_cuda and parent.is_cuda
    g, parent = g.cpu().numpy(), parent.cpu().numpy()
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("device", g, parent, off[i], pr, fin.g, fin.parent)


def test_batch_iteration_cap(P):
    probs = problem_set()[:3]
    B = build(P, probs, max_iters=2)
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs),
                                allow_not_converged=True)
    assert stats[0]["rc"] == P.PIRRT_ENOTCONVERGED
    off = B.offsets
    capped = 0
    for i, pr in enumerate(probs):
        R = O.Graph()
        assert R.insert_batch(W.Batch(0, pr.n, *pr.rows, 0.0)) == 0
        rc, st = R.replan(pr.root, pr.goal, pr.h, True, max_iters=2)
        capped += rc != 0
        fin = R.state()
        check_problem("cap", g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k)
    assert capped > 0


def test_batch_invalid_arguments(P):
    probs = problem_set()[:2]
    B = build(P, probs)
    n0 = B.n
    # a neighbour at or beyond the row's own local id
    bad = (np.array([0, 0, 1], np.int64), np.array([1], np.int32), np.array([1.0], np.float32))
    with pytest.raises(P.PirrtError):
        B.add_problem(*bad)
    with pytest.raises(P.PirrtError):
        B.add_problem(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert B.num_problems == 2 and B.n == n0
    with pytest.raises(P.PirrtError):
        B.replan([0, probs[1].n], [1, 1])
    with pytest.raises(ValueError):
        B.replan([0], [1])
    # still usable
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("after errors", g, parent, B.offsets[i], pr, fin.g, fin.parent)


def test_batch_tune(P):
    probs = problem_set()[:6]
    B = build(P, probs)
    cfg = B.tune([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    assert 0 <= cfg < 32  # row split + 4 x stamp scope + 8 x grid-size index
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    off = B.offsets
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("tuned", g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k)


@pytest.mark.parametrize("blocks", [1, 7, 1024, 8192])
def test_batch_grid_sizes(P, monkeypatch, blocks):
    """The batch kernels stride over the live work with any number of workgroups,
    down to one: the results and counters stay the oracle's."""
    monkeypatch.setenv("PIRRT_BATCH_BLOCKS", str(blocks))
    probs = problem_set()
    B = build(P, probs)
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    off = B.offsets
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("blocks %d" % blocks, g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k, blocks)


@pytest.mark.parametrize("bitmap_tiles", [0])
def test_batch_tile_list_without_bitmap(P, monkeypatch, bitmap_tiles):
    """The active tile list taken tile by tile (the path for batches with more tiles
    than the LDS bitmap holds) gives the oracle's results and counters too."""
    monkeypatch.setenv("PIRRT_TILE_BITMAP", str(bitmap_tiles))
    probs = problem_set()
    B = build(P, probs)
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs))
    off = B.offsets
    for i, pr in enumerate(probs):
        _, rc, st, fin = oracle_run(pr)
        check_problem("tile list %d" % bitmap_tiles, g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k, bitmap_tiles)


def test_batch_phase_timing(P):
    """With timing on, every problem's entry holds the batch's phase times; the
    results stay those of the oracle."""
    probs = problem_set()
    B = build(P, probs)
    off = B.offsets
    B.snapshot_save()
    roots, goals = [p.root for p in probs], [p.goal for p in probs]
    g, parent, stats = B.replan(roots, goals, full_h(probs), timing=True)
    want = [oracle_run(pr) for pr in probs]
    for i, pr in enumerate(probs):
        check_problem("timed", g, parent, off[i], pr, want[i][3].g, want[i][3].parent)
    first = stats[0]
    assert first["ms_improve"] > 0 and first["ms_evaluate"] > 0 and first["ms_mark"] > 0
    # one Improve launch per loop iteration of the batch: the longest problem's count
    assert first["improve_launches"] == max(s["iterations"] for s in stats)
    for s in stats[1:]:
        for k in ("ms_evaluate", "ms_mark", "ms_improve", "improve_launches", "mark_launches", "evaluate_calls"):
            assert s[k] == first[k], k


def test_batch_lookahead_matches_single_problems(P):
    """The narrowed Improve domain on a batch: every problem ends where the oracle's
    narrowed mode ends on that problem alone."""
    probs = problem_set()
    B = build(P, probs)
    off = B.offsets
    g, parent, stats = B.replan([p.root for p in probs], [p.goal for p in probs], full_h(probs), lookahead=True)
    for i, pr in enumerate(probs):
        R = O.Graph()
        rp, col, cst = pr.rows
        assert R.insert_batch(W.Batch(0, pr.n, rp, col, cst, 0.0)) == 0
        rc, st = R.replan(pr.root, pr.goal, pr.h, pr.prune, lookahead=True)
        fin = R.state()
        assert rc == 0 and stats[i]["rc"] == 0
        check_problem("lookahead", g, parent, off[i], pr, fin.g, fin.parent)
        for k in STAT_KEYS:
            assert stats[i][k] == st[k], (pr.name, k, stats[i][k], st[k])
