"""Parity at the full workload sizes: the 6D batched-extension run (100 batches of
1,000 vertices, Replan after every batch) and the 6D 1,000,000-vertex graph (one
Replan from the insertion-time policy, then a further 10,000-vertex batch and a
second Replan; the benchmark's timed path of repeated Replans from captured loop
graphs) and the 512-problem batched set, every problem against the oracle."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import assert_same_policy, assert_same_stats, gpu_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


def test_berrt_6d_100k(P):
    wl = W.batched_6d(batches=100, batch=1000, seed=100)
    G = gpu_graph(P)
    R = O.Graph()
    for i, b in enumerate(wl.batches):
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
        h = wl.heuristic(G.n)
        gg, pp, sg = G.replan(0, 1, h, True)
        rc, so = R.replan(0, 1, h, True)
        assert rc == 0
        st = R.state()
        assert_same_policy("batch %d" % i, gg, pp, st.g, st.parent)
        assert_same_stats("batch %d" % i, sg, so)
    print("100k: n=%d nnz=%d" % (G.n, G.nnz), flush=True)


@pytest.fixture(scope="module")
def big():
    return W.plain_6d(samples=1_000_000, extra=10_000, seed=200)


def test_plain_6d_1m(P, big):
    wl = big
    G = gpu_graph(P)
    R = O.Graph()
    b0, b1 = wl.batches
    G.insert_rows(b0)
    assert R.insert_batch(b0) == 0
    g, p, c = G.get_policy()
    st = R.state()
    assert_same_policy("insert 1M", g, p, st.g, st.parent)
    h = wl.heuristic(G.n)
    gg, pp, sg = G.replan(0, 1, h, True)
    rc, so = R.replan(0, 1, h, True)
    assert rc == 0
    st = R.state()
    assert_same_policy("replan 1M", gg, pp, st.g, st.parent)
    assert_same_stats("replan 1M", sg, so)
    print("1M replan stats", sg, flush=True)
    G.insert_rows(b1)
    assert R.insert_batch(b1) == 0
    g, p, c = G.get_policy()
    st = R.state()
    assert_same_policy("insert +10k", g, p, st.g, st.parent)
    h = wl.heuristic(G.n)
    gg, pp, sg = G.replan(0, 1, h, True)
    rc, so = R.replan(0, 1, h, True)
    assert rc == 0
    st = R.state()
    assert_same_policy("replan +10k", gg, pp, st.g, st.parent)
    assert_same_stats("replan +10k", sg, so)
    print("+10k replan stats", sg, flush=True)


def test_plain_6d_1m_timed_path(P, big):
    """The benchmark's timed path at full size: the 1M-vertex graph on the caller's
    stream, the autotuner's configuration, then repeated Replans from the restored
    insertion-time policy into device buffers.  The second call with the same
    arguments captures the loop bodies as HIP graphs and the third replays them;
    every call's g (bit for bit), parents and counters must equal the oracle's."""
    import torch
    wl = big
    dev = torch.device("cuda:0")
    G = gpu_graph(P, device=0)
    b0 = wl.batches[0]
    G.insert_rows(b0)
    G.snapshot_save()
    n = G.n
    hh = wl.heuristic(n)
    h = torch.from_numpy(hh).to(dev)
    g_out = torch.empty(n, dtype=torch.float32, device=dev)
    p_out = torch.empty(n, dtype=torch.int32, device=dev)
    config = G.tune(0, 1, h, True)
    R = O.Graph()
    assert R.insert_batch(b0) == 0
    rc, so = R.replan(0, 1, hh, True)
    assert rc == 0
    st = R.state()
    for call in range(3):
        G.snapshot_restore()
        _, _, sg = G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out)
        tag = "1M call %d (configuration %d)" % (call, config)
        assert_same_policy(tag, g_out.cpu().numpy(), p_out.cpu().numpy(), st.g, st.parent)
        assert_same_stats(tag, sg, so)
    print("1M timed path: configuration %d, %d iterations" % (config, so["iterations"]), flush=True)


def test_truncated_6d_1m(P, big):
    """The truncated Evaluate at full size: the Replan, the +10k batch inserted on top of
    the stale g it leaves (the insertion-time policy compared too), the second Replan."""
    wl = big
    G = gpu_graph(P)
    R = O.Graph()
    for i, b in enumerate(wl.batches):
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
        if i > 0:
            g, p, c = G.get_policy()
            st = R.state()
            assert_same_policy("insert %d after truncated Replan" % i, g, p, st.g, st.parent)
        h = wl.heuristic(G.n)
        gg, pp, sg = G.replan(0, 1, h, True, truncated=True)
        rc, so = R.replan(0, 1, h, True, truncated=True)
        assert rc == 0
        st = R.state()
        assert_same_policy("truncated replan %d" % i, gg, pp, st.g, st.parent)
        assert_same_stats("truncated replan %d" % i, sg, so)
        print("truncated replan %d stats" % i, sg, flush=True)


def _oracle_problem(rows, h, root, goal):
    """One problem replanned by the oracle on rows given as (row_ptr, col, cost)."""
    orc = O.Graph()
    assert orc.insert(*rows) == 0
    rc, so = orc.replan(root, goal, h, True)
    st = orc.state()
    return rc, so, st.g, st.parent


def test_multi_graph_512(P):
    """The 512-problem multi-graph set (28.6M vertices) built on the device and
    replanned by one batched call, as the benchmark's multi workload does.  Every
    problem is compared with the oracle run on that problem alone: the oracle reads
    the problem's rows and heuristic as the device built them (the device builder's
    rows and heuristic equal the exploration oracle's bit for bit, which
    test_gpu_rrg.py checks), and the g bits, parents and counters must be equal.
    Eight problems of different dimensions are also rebuilt from scratch by the
    exploration oracle (points, rows, heuristic) to tie the chain end to end."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    from oracle import rrg as RR
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    specs = [W.multi_problem_spec(i) for i in range(512)]
    B = P.Batch(stream=stream)
    hs, rrgs = [], []
    for sp in specs:
        R = P.Rrg(sp.d, sp.obstacles, stream=stream, point_capacity=sp.n)
        R.add_points(np.stack([np.full(sp.d, 0.05), np.full(sp.d, 0.95)]))
        R.sample(sp.sample_seed, 0, 0, sp.n - 2)
        R.connect_problem(sp.radius, B)
        hs.append(R.heuristic(1, out=torch.empty(sp.n, dtype=torch.float32, device=dev)))
        rrgs.append(R)
    print("built %d problems: n=%d nnz=%d" % (len(specs), B.n, B.nnz), flush=True)
    h = torch.cat(hs)
    g, parent, stats = B.replan(np.zeros(512, np.int32), np.ones(512, np.int32), h)
    g, parent = g.cpu().numpy(), parent.cpu().numpy()
    assert all(s["rc"] == 0 for s in stats)
    off = B.offsets
    hh = h.cpu().numpy()
    # every problem against the oracle, several problems at a time on the host's
    # cores (the oracle runs in C and releases the interpreter lock)
    try:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    except (AttributeError, OSError):
        workers = max(1, min(16, os.cpu_count() or 1))
    order = sorted(range(512), key=lambda i: -specs[i].n)  # largest first: better packing
    done = 0
    with ThreadPoolExecutor(max_workers=workers) as ex:
        pending = []

        def drain(limit):
            nonlocal done
            while len(pending) > limit:
                i, fut = pending.pop(0)
                rc, so, go, po = fut.result()
                assert rc == 0, i
                tag = "problem %d (d=%d n=%d)" % (i, specs[i].d, specs[i].n)
                assert_same_policy(tag, g[off[i]:off[i + 1]], parent[off[i]:off[i + 1]], go, po)
                assert_same_stats(tag, stats[i], so)
                done += 1

        for i in order:
            rows = rrgs[i].rows(0, specs[i].radius)
            pending.append((i, ex.submit(_oracle_problem, rows, hh[off[i]:off[i + 1]], 0, 1)))
            drain(2 * workers)
        drain(0)
    assert done == 512
    print("all 512 problems equal the oracle (%d host threads)" % workers, flush=True)
    # invariants on every problem (device arithmetic: binary32 adds, no contraction)
    gd, pd, cd = B.get_policy(device=dev)
    base = torch.from_numpy(np.repeat(off[:-1], np.diff(off))).to(dev)
    has = pd >= 0
    gp = gd[(pd.long() + base)[has]]
    assert torch.equal((gp + cd[has]).view(torch.int32), gd[has].view(torch.int32))
    assert torch.all(gd[torch.from_numpy(off[:-1]).to(dev)] == 0)
    # sampled problems against the oracle's own build
    picked, seen = [], set()
    for sp in specs:
        if sp.n <= 12000 and (sp.d, sp.n > 8000) not in seen:
            seen.add((sp.d, sp.n > 8000))
            picked.append(sp)
        if len(picked) == 8:
            break
    for sp in picked:
        i = sp.index
        pts = np.concatenate([np.stack([np.full(sp.d, 0.05), np.full(sp.d, 0.95)]),
                              RR.sample(sp.d, sp.sample_seed, 0, 0, sp.n - 2, sp.obstacles)[0]])
        assert np.array_equal(rrgs[i].points(), pts)
        rp, col, cost = RR.build_rows(pts, 0, sp.radius, sp.obstacles)
        orc = O.Graph()
        assert orc.insert_batch(W.Batch(0, sp.n, rp, col, cost, sp.radius)) == 0
        rc, so = orc.replan(0, 1, RR.heuristic(pts, pts[1]), True)
        assert rc == 0
        st = orc.state()
        assert_same_policy("problem %d (d=%d n=%d)" % (i, sp.d, sp.n), g[off[i]:off[i + 1]],
                           parent[off[i]:off[i + 1]], st.g, st.parent)
        assert_same_stats("problem %d" % i, stats[i], so)
    print("compared problems %s with the oracle's own build" % [sp.index for sp in picked], flush=True)
