"""The rest of the C ABI around Replan, through ctypes, against the oracle:

- pirrt_batch_insert: problems of a batch grow by batches of vertices (Alg. 3's
  exploration step for many planners) with a batched Replan after every round; each
  problem must end exactly where the oracle ends on a graph holding that problem
  alone after the same inserts and Replans (g bit for bit, parents, statistics).
- pirrt_state_save / pirrt_state_restore: a checkpoint blob restores the saved graph
  and policy into a fresh handle, whose next Replan equals the oracle's.
- allocator callbacks: a graph whose device memory comes from torch's caching
  allocator replans exactly like the oracle and returns every block at destroy."""
import numpy as np
import pytest

import oracle as O
import workloads as W

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


def growing_problems(count, rounds, seed):
    """count problems of dimensions 2-6, each a workload of `rounds` batches of
    uneven sizes (some rounds add nothing to some problems)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = [2, 3, 4, 6][i % 4]
        obs = W.make_obstacles(d, int(rng.integers(4, 20)), "mixed", seed + 10 * i)
        sizes = [int(rng.integers(40, 400)) for _ in range(rounds)]
        for r in range(1, rounds):
            if rng.random() < 0.2:
                sizes[r] = 0
        sizes = [s for s in sizes]
        nz = [s for s in sizes if s > 0]
        wl = W.grow("grow-%d" % i, d, obs, seed + 10 * i + 1, nz)
        # map each round to its batch (None for an empty round)
        it = iter(wl.batches)
        per_round = [next(it) if s > 0 else None for s in sizes]
        out.append((wl, per_round))
    return out


def concat(blocks):
    ptr = [np.zeros(1, np.int64)]
    cols, costs, base = [], [], 0
    for b in blocks:
        ptr.append(b.row_ptr[1:].astype(np.int64) + base)
        cols.append(b.col.astype(np.int32))
        costs.append(b.cost.astype(np.float32))
        base += int(b.row_ptr[-1])
    return np.concatenate(ptr), np.concatenate(cols), np.concatenate(costs)


def test_batch_grows_problems_over_rounds(P):
    import torch
    probs = growing_problems(16, 5, seed=5150)
    B = P.Batch(stream=torch.cuda.current_stream().cuda_stream)
    refs = []
    for wl, rounds in probs:
        first = rounds[0]
        B.add_problem(first.row_ptr, first.col, first.cost)
        R = O.Graph()
        assert R.insert_batch(first) == 0
        refs.append(R)
    rng = np.random.default_rng(7)
    for r in range(5):
        if r > 0:
            order = [int(i) for i in rng.permutation(len(probs))]
            grown = [i for i in order if probs[i][1][r] is not None]
            skipped = [i for i in order if probs[i][1][r] is None]
            # a listed problem with no rows, and problems in shuffled order
            listed = grown + skipped[:1]
            blocks = [probs[i][1][r] for i in grown]
            n_new = [probs[i][1][r].n_new for i in grown] + [0] * len(skipped[:1])
            rp, col, cost = concat(blocks)
            B.insert(listed, n_new, rp, col, cost)
            for i in grown:
                assert refs[i].insert_batch(probs[i][1][r]) == 0
        ns = [R.n for R in refs]
        assert B.num_problems == len(probs)
        assert [B.problem_offset(i) for i in range(len(probs) + 1)] == list(np.concatenate([[0], np.cumsum(ns)]))
        h = np.concatenate([probs[i][0].heuristic(ns[i]) for i in range(len(probs))]).astype(np.float32)
        g, parent, stats = B.replan([0] * len(probs), [1] * len(probs), h, True)
        for i, R in enumerate(refs):
            a, b = B.problem_offset(i), B.problem_offset(i + 1)
            hi = h[a:b]
            rc, so = R.replan(0, 1, hi, True)
            assert rc == 0
            ref = R.state()
            assert np.array_equal(g[a:b].view(np.uint32), ref.g.view(np.uint32)), (r, i)
            assert np.array_equal(parent[a:b], ref.parent), (r, i)
            for k in STAT_KEYS:
                assert stats[i][k] == so[k], (r, i, k)


def test_batch_insert_rejects_bad_calls(P):
    import torch
    wl = W.grow("g", 2, W.make_obstacles(2, 4, "box", 3), 4, [100, 50])
    B = P.Batch(stream=torch.cuda.current_stream().cuda_stream)
    for _ in range(2):
        B.add_problem(wl.batches[0].row_ptr, wl.batches[0].col, wl.batches[0].cost)
    b = wl.batches[1]
    before = B.get_policy()
    for problems, n_new, col in (([0, 0], [b.n_new, 0], b.col),      # repeated problem
                                 ([2], [b.n_new], b.col),            # out of range
                                 ([1], [b.n_new], b.col + 10_000)):   # neighbour beyond its own id
        rp, c, cost = concat([W.Batch(b.n_old, b.n_new, b.row_ptr, col.astype(np.int32), b.cost, b.radius)])
        with pytest.raises(P.PirrtError) as e:
            B.insert(problems, n_new, rp, c, cost)
        assert e.value.code == P.PIRRT_EINVAL
    after = B.get_policy()
    assert B.n == 2 * wl.batches[0].n_new
    for x, y in zip(before, after):
        assert np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32))
    # and the batch still grows afterwards
    B.insert([1], [b.n_new], b.row_ptr, b.col, b.cost)
    assert B.problem_offset(2) == 2 * wl.batches[0].n_new + b.n_new


def test_state_blob_round_trip(P):
    import torch
    wl = W.batched_6d(batches=3, batch=700, seed=321)
    G = P.Graph(stream=torch.cuda.current_stream().cuda_stream)
    R = O.Graph()
    for b in wl.batches[:2]:
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
    h = wl.heuristic(G.n)
    G.replan(0, 1, h, True)
    assert R.replan(0, 1, h, True)[0] == 0
    saved = G.get_policy()
    blob = G.state_save()
    assert blob.size == G.state_size()
    # a fresh handle from the blob holds the same graph and policy
    G2 = P.Graph(stream=torch.cuda.current_stream().cuda_stream)
    G2.state_restore(blob)
    assert G2.n == G.n and G2.nnz == G.nnz
    for x, y in zip(saved, G2.get_policy()):
        assert np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32))
    ref = R.state()
    assert np.array_equal(saved[0].view(np.uint32), ref.g.view(np.uint32))
    assert np.array_equal(saved[1], ref.parent)
    a1, a2 = G.adjacency(), G2.adjacency()
    assert np.array_equal(a1[0], a2[0])
    for v in range(0, G.n, 97):  # rows hold the same neighbours and costs (order free)
        r1 = sorted(zip(a1[1][a1[0][v]:a1[0][v + 1]], a1[2][a1[0][v]:a1[0][v + 1]].view(np.uint32)))
        r2 = sorted(zip(a2[1][a2[0][v]:a2[0][v + 1]], a2[2][a2[0][v]:a2[0][v + 1]].view(np.uint32)))
        assert r1 == r2, v
    # both continue like the oracle: a further batch and Replan
    b = wl.batches[2]
    G2.insert_rows(b)
    assert R.insert_batch(b) == 0
    h = wl.heuristic(G2.n)
    g, parent, st = G2.replan(0, 1, h, True)
    rc, so = R.replan(0, 1, h, True)
    ref = R.state()
    assert np.array_equal(g.view(np.uint32), ref.g.view(np.uint32))
    assert np.array_equal(parent, ref.parent)
    for k in STAT_KEYS:
        assert st[k] == so[k], k
    # policy-only restore into the handle that holds the saved graph
    G.set_policy(np.zeros(G.n, np.float32), np.full(G.n, -1, np.int32), np.zeros(G.n, np.float32))
    G.state_restore(blob)
    for x, y in zip(saved, G.get_policy()):
        assert np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32))
    # a handle holding another graph, a truncated blob and a foreign blob are refused
    for bad in (blob[:100], np.zeros_like(blob)):
        with pytest.raises(P.PirrtError) as e:
            G2.state_restore(bad)
        assert e.value.code == P.PIRRT_EINVAL
    with pytest.raises(P.PirrtError) as e:
        G2.state_restore(blob)  # G2 grew since
    assert e.value.code == P.PIRRT_EINVAL


def test_allocator_callbacks_use_torch_cache(P):
    import torch
    wl = W.plain_2d(samples=3000, seed=9)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    G = P.Graph(stream=torch.cuda.current_stream().cuda_stream, torch_allocator=True)
    R = O.Graph()
    for b in wl.batches:
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
    held = torch.cuda.memory_allocated() - base
    assert held > 0, "the graph's storage did not come from torch's allocator"
    h = wl.heuristic()
    g, parent, st = G.replan(0, 1, h, True)
    rc, so = R.replan(0, 1, h, True)
    ref = R.state()
    assert rc == 0
    assert np.array_equal(g.view(np.uint32), ref.g.view(np.uint32))
    assert np.array_equal(parent, ref.parent)
    G.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base, "blocks not returned at destroy"
