"""Parity at the full workload sizes: the 6D batched-extension run (100 batches of
1,000 vertices, Replan after every batch) and the 6D 1,000,000-vertex graph (one
Replan from the insertion-time policy, then a further 10,000-vertex batch and a
second Replan), in the same launch configuration the benchmark times."""
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
