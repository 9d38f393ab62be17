"""Device-side RRG construction (pirrt_rrg_* through the C ABI) against the
exploration-support oracle: sampled points, rows, costs and heuristic bit for bit,
and Replan on a device-built graph against the oracle on its own build."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import rrg as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


def stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


ROOT_GOAL = lambda d: np.stack([np.full(d, 0.05), np.full(d, 0.95)])


@pytest.mark.parametrize("d,count,kinds", [(1, 3, "sphere"), (2, 8, "box"), (3, 12, "mixed"), (4, 20, "sphere"),
                                           (5, 10, "box"), (6, 40, "sphere"), (7, 20, "mixed"), (8, 15, "mixed")])
def test_sample_rows_heuristic(P, d, count, kinds):
    obs = W.make_obstacles(d, count, kinds, 17 * d)
    n = 1500 if d <= 6 else 900
    G = P.Rrg(d, obs, stream=stream())
    G.add_points(ROOT_GOAL(d))
    c1 = G.sample(seed=77, stream=d, counter=0, count=n // 2)
    c2 = G.sample(seed=77, stream=d, counter=c1, count=n - n // 2)
    want, wc = R.sample(d, 77, d, 0, n, obs)
    pts = G.points()
    assert c2 == wc
    assert np.array_equal(pts[2:], want)
    r = W.radius(n + 2, d)
    rp, col, cost = G.rows(0, r)
    orp, ocol, ocost = R.build_rows(pts, 0, r, obs)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    assert np.array_equal(cost.view(np.uint32), ocost.view(np.uint32))
    k = n // 4  # the rows of a later batch
    rp2, col2, cost2 = G.rows(n + 2 - k, r)
    orp2, ocol2, ocost2 = R.build_rows(pts, n + 2 - k, r, obs)
    assert np.array_equal(rp2, orp2) and np.array_equal(col2, ocol2)
    assert np.array_equal(cost2.view(np.uint32), ocost2.view(np.uint32))
    h = G.heuristic(1)
    assert np.array_equal(h.view(np.uint32), R.heuristic(pts, pts[1]).view(np.uint32))
    # the same rows into device buffers: room enough, and too little room (one retry)
    import torch
    for cap in (None, 3):
        drp, dcol, dcost = G.rows(n + 2 - k, r, device=torch.device("cuda:0"), capacity=cap)
        assert np.array_equal(drp.cpu().numpy(), orp2) and np.array_equal(dcol.cpu().numpy(), ocol2)
        assert np.array_equal(dcost.cpu().numpy().view(np.uint32), ocost2.view(np.uint32))


def test_connect_and_replan_in_batches(P):
    """BERRT#-style growth: batches sampled and connected on the device, Replan
    after each; the oracle builds its own graph from its own rows."""
    d = 6
    obs = W.make_obstacles(d, 40, "sphere", 100)
    G = P.Rrg(d, obs, stream=stream())
    G.add_points(ROOT_GOAL(d))
    graph = P.Graph(stream=stream())
    orc = O.Graph()
    counter, n_old = 0, 0
    for b in range(5):
        counter = G.sample(seed=3, stream=0, counter=counter, count=400)
        n = G.n
        r = W.radius(n, d)
        G.connect(n_old, r, graph)
        opts = np.concatenate([ROOT_GOAL(d), R.sample(d, 3, 0, 0, n - 2, obs)[0]])
        rp, col, cost = R.build_rows(opts, n_old, r, obs)
        assert orc.insert_batch(W.Batch(n_old, n - n_old, rp, col, cost, r)) == 0
        h = R.heuristic(opts, opts[1])
        hd = G.heuristic(1)
        assert np.array_equal(hd.view(np.uint32), h.view(np.uint32))
        gg, pp, sg = graph.replan(0, 1, hd, True)
        rc, so = orc.replan(0, 1, h, True)
        st = orc.state()
        assert rc == 0 and np.array_equal(gg.view(np.uint32), st.g.view(np.uint32))
        assert np.array_equal(pp, st.parent)
        for k in ("iterations", "edges_examined", "sum_P", "sum_D", "changed_total", "mark_edges"):
            assert sg[k] == so[k], (b, k)
        n_old = n
    assert np.array_equal(G.points(), opts)


def test_connect_problem_into_batch(P):
    B = P.Batch(stream=stream())
    probs = []
    for i, (d, kinds) in enumerate([(2, "box"), (4, "mixed"), (6, "sphere"), (8, "mixed"), (3, "sphere")]):
        obs = W.make_obstacles(d, 12, kinds, 500 + i)
        G = P.Rrg(d, obs, stream=stream())
        G.add_points(ROOT_GOAL(d))
        G.sample(seed=1000 + i, stream=0, counter=0, count=600 + 150 * i)
        r = W.radius(G.n, d)
        assert G.connect_problem(r, B) == i
        pts = G.points()
        probs.append((pts, r, obs, G.heuristic(1)))
    off = B.offsets
    h = np.concatenate([p[3] for p in probs])
    g, parent, stats = B.replan([0] * len(probs), [1] * len(probs), h)
    for i, (pts, r, obs, hp) in enumerate(probs):
        rp, col, cost = R.build_rows(pts, 0, r, obs)
        orc = O.Graph()
        assert orc.insert_batch(W.Batch(0, len(pts), rp, col, cost, r)) == 0
        rc, so = orc.replan(0, 1, R.heuristic(pts, pts[1]), True)
        st = orc.state()
        assert rc == 0
        assert np.array_equal(g[off[i]:off[i + 1]].view(np.uint32), st.g.view(np.uint32))
        assert np.array_equal(parent[off[i]:off[i + 1]], st.parent)
        assert stats[i]["edges_examined"] == so["edges_examined"]


def test_rrg_invalid_arguments(P):
    obs = W.make_obstacles(3, 4, "mixed", 1)
    with pytest.raises(P.PirrtError):
        P.Rrg(9, None)
    G = P.Rrg(3, obs, stream=stream())
    with pytest.raises(P.PirrtError):
        G.add_points(np.array([[0.1, np.nan, 0.2]]))
    assert G.n == 0
    G.add_points(ROOT_GOAL(3))
    with pytest.raises(P.PirrtError):
        G.rows(0, -1.0)
    with pytest.raises(P.PirrtError):
        G.heuristic(5)
    graph = P.Graph(stream=stream())
    with pytest.raises(P.PirrtError):
        G.connect(1, 0.3, graph)  # the graph holds 0 points, not 1
    G.connect(0, 0.3, graph)
    assert graph.n == 2


@pytest.mark.parametrize("n_cand,count", [(8192, 500), (1000, 1000), (777, 13)])
def test_sample_learned(P, n_cand, count):
    """The learned sampler appends exactly the `count` best-scored of the oracle's
    n_cand free candidates (the network's own logits, ties to the earlier
    candidate), in candidate order, and advances the counter past them."""
    from oracle import mlp as ML
    d = 6
    obs = W.make_obstacles(d, 40, "sphere", 77)
    enc = ML.obstacle_encoding(obs).astype(np.float32)
    net = P.Mlp(d + len(enc), 8192)
    p = ML.init_params(np.random.default_rng(3), d + len(enc))
    net.set_params(np.concatenate([np.asarray(getattr(p, k), np.float32).ravel() for k in ML.PARAM_NAMES]))
    G = P.Rrg(d, obs, stream=stream())
    G.add_points(ROOT_GOAL(d))
    c = G.sample_learned(net, enc, seed=5, stream=9, counter=0, n_candidates=n_cand, count=count)
    cand, want_c = R.sample(d, 5, 9, 0, n_cand, obs)
    assert c == want_c
    feats = np.concatenate([cand.astype(np.float32), np.broadcast_to(enc, (n_cand, len(enc)))], axis=1)
    logits = net.forward(np.ascontiguousarray(feats, np.float32))
    order = np.lexsort((np.arange(n_cand), -logits.astype(np.float64)))
    chosen = np.sort(order[:count])
    got = G.points(2)
    assert np.array_equal(got, cand[chosen])
    with pytest.raises(P.PirrtError):
        G.sample_learned(net, enc[:-1], seed=5, stream=9, counter=0, n_candidates=10, count=5)
