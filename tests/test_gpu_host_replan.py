"""The adaptive CPU/GPU placement of pirrt_replan (small graphs replan on the host,
csrc/host_replan.hip) against the oracle: the host path must give the oracle's g bit
for bit, its parents and its counters, exactly as the device loop does, and the
handle must move between the two as the graph grows without any difference showing.
The host path is forced on larger graphs too (PIRRT_HOST_MAX) so that it meets the
same cases as the device loop."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle_pins import fixtures, load_fixture
from test_gpu_parity import assert_same_policy, assert_same_stats, lattice_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


def graph(P, **kw):
    import torch
    return P.Graph(stream=torch.cuda.current_stream().cuda_stream, **kw)


def both(P, batches, plan, h_of=None, prune=True, lookahead=False, expect_host=True, **kw):
    G = graph(P, **kw)
    R = O.Graph()
    for i, b in enumerate(batches):
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
        if i in plan:
            root, goal = plan[i]
            h = None if h_of is None else h_of(G.n)
            gg, pp, sg = G.replan(root, goal, h, prune, lookahead=lookahead)
            rc, so = R.replan(root, goal, h, prune, lookahead=lookahead)
            assert rc == 0
            assert sg["on_host"] == (1 if expect_host else 0), (i, G.n)
            st = R.state()
            assert_same_policy("host replan %d" % i, gg, pp, st.g, st.parent)
            assert_same_stats("host replan %d" % i, sg, so)
    return G, R


@pytest.fixture
def host_always(monkeypatch):
    monkeypatch.setenv("PIRRT_HOST_MAX", "100000000")


def test_golden_fixtures_on_host(P, host_always):
    for path in fixtures():
        fx = load_fixture(path)
        G = graph(P)
        G.insert_rows(W.from_edges(fx["n"], fx["edges"]))
        gg, pp, st = G.replan(fx["root"], fx["goal"], fx["h"], bool(fx["prune"]))
        assert st["on_host"] == 1
        assert np.array_equal(gg, fx["expect_g"]), (path, gg)
        assert np.array_equal(pp, fx["expect_parent"]), (path, pp)
        for k, v in fx["expect_stats"].items():
            assert st[k] == v, (path, k, st[k], v)


@pytest.mark.parametrize("prune,lookahead", [(True, False), (False, False), (True, True)])
def test_plain_2d_on_host(P, host_always, prune, lookahead):
    wl = W.plain_2d()
    both(P, wl.batches, {0: (0, 1)}, wl.heuristic, prune, lookahead)


def test_batched_6d_on_host(P, host_always):
    wl = W.batched_6d(batches=8, batch=400, seed=100)
    both(P, wl.batches, {i: (0, 1) for i in range(8)}, wl.heuristic, True)


@pytest.mark.parametrize("prune", [True, False])
def test_lattice_ties_on_host(P, host_always, prune):
    both(P, [lattice_batch(30, 0.85, 12)], {0: (0, 1)}, None, prune)


def test_iteration_cap_on_host(P, host_always):
    wl = W.plain_2d(samples=800, seed=4)
    G = graph(P, max_iters=2)
    R = O.Graph()
    G.insert_rows(wl.batches[0])
    R.insert_batch(wl.batches[0])
    gg, pp, sg = G.replan(0, 1, wl.heuristic(), True, allow_not_converged=True)
    rc, so = R.replan(0, 1, wl.heuristic(), True, max_iters=2)
    assert sg["rc"] == P.PIRRT_ENOTCONVERGED and rc == O.ENOTCONVERGED and sg["on_host"] == 1
    st = R.state()
    assert_same_policy("cap", gg, pp, st.g, st.parent)
    assert_same_stats("cap", sg, so)


def test_degenerate_and_orphans_on_host(P, host_always):
    edges = [(0, 2, 0.0), (2, 3, 1.0), (4, 5, 1.0), (5, 6, 0.5), (3, 1, 2.0)]
    b = W.from_edges(8, edges)
    G, R = both(P, [b], {0: (0, 1)}, None, True)
    for prune in (True, False):
        gg, pp, sg = G.replan(0, 1, None, prune)
        rc, so = R.replan(0, 1, None, prune)
        st = R.state()
        assert_same_policy("degenerate", gg, pp, st.g, st.parent)
        assert_same_stats("degenerate", sg, so)
    wl = W.plain_2d(samples=600, seed=3)
    G = graph(P)
    R = O.Graph()
    G.insert_rows(wl.batches[0])
    R.insert_batch(wl.batches[0])
    n = G.n
    z = (np.full(n, np.inf, np.float32), np.full(n, -1, np.int32), np.zeros(n, np.float32))
    G.set_policy(*z)
    R.set_state(*z)
    gg, pp, sg = G.replan(0, 1, wl.heuristic(), True)
    rc, so = R.replan(0, 1, wl.heuristic(), True)
    st = R.state()
    assert_same_policy("orphans", gg, pp, st.g, st.parent)
    assert_same_stats("orphans", sg, so)


def test_new_roots_and_device_buffers_on_host(P, host_always):
    """Root marks move between calls; device h and outputs; the device arrays stay the
    handle's state (a snapshot of them restores and replans the same way)."""
    import torch
    wl = W.batched_6d(batches=1, batch=900, seed=104)
    G = graph(P)
    R = O.Graph()
    b = wl.batches[0]
    G.insert_rows(b)
    assert R.insert_batch(b) == 0
    n = G.n
    h = wl.heuristic(n)
    hd = torch.from_numpy(h).cuda()
    k = n // 2
    for call, (root, goal) in enumerate([(0, 1), (k, 1), (0, 1)]):
        gg, pp, sg = G.replan(root, goal, hd, True)
        assert gg.is_cuda and sg["on_host"] == 1
        rc, so = R.replan(root, goal, h, True)
        assert rc == 0
        st = R.state()
        assert_same_policy("call %d" % call, gg.cpu().numpy(), pp.cpu().numpy(), st.g, st.parent)
        assert_same_stats("call %d" % call, sg, so)
    g1, p1, c1 = G.get_policy()
    st = R.state()
    assert_same_policy("stored", g1, p1, st.g, st.parent)
    assert np.array_equal(c1.view(np.uint32), st.pcost.view(np.uint32))


def test_placement_follows_size(P, monkeypatch):
    """Default threshold: the handle replans on the host while the graph is small and
    on the device once it has grown past 512 vertices; every Replan equals the
    oracle's.  PIRRT_HOST_MAX=0 keeps even the smallest graph on the device."""
    monkeypatch.delenv("PIRRT_HOST_MAX", raising=False)
    wl = W.grow("placement", 2, W.make_obstacles(2, 6, "box", 31), 32, [60, 150, 200, 300, 500])
    G = graph(P)
    R = O.Graph()
    places = []
    for b in wl.batches:
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
        h = wl.heuristic(G.n)
        gg, pp, sg = G.replan(0, 1, h, True)
        rc, so = R.replan(0, 1, h, True)
        st = R.state()
        assert_same_policy("n=%d" % G.n, gg, pp, st.g, st.parent)
        assert_same_stats("n=%d" % G.n, sg, so)
        places.append((G.n, sg["on_host"]))
    assert all(on == (1 if n <= 512 else 0) for n, on in places), places
    assert any(on for _, on in places) and not all(on for _, on in places)
    monkeypatch.setenv("PIRRT_HOST_MAX", "0")
    G0 = graph(P)
    G0.insert_rows(wl.batches[0])
    _, _, s0 = G0.replan(0, 1, wl.heuristic(G0.n), True)
    assert s0["on_host"] == 0
