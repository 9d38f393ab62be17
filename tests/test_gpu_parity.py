"""GPU Replan (libpirrt.so through its C ABI) against the oracle, element by element.

g must match bit for bit (compared as uint32), parents exactly, and the
per-Replan statistics (iterations, |P| and |D| sums, edges examined, parents
switched) exactly: the GPU path follows the same algorithm step by step.
"""
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


@pytest.fixture(autouse=True)
def device_path(monkeypatch):
    """These cases test the device loop: small graphs stay on the device too."""
    monkeypatch.setenv("PIRRT_HOST_MAX", "0")


def gpu_graph(P, **kw):
    import torch
    return P.Graph(stream=torch.cuda.current_stream().cuda_stream, **kw)


def assert_same_policy(tag, g_gpu, p_gpu, g_orc, p_orc):
    g_gpu = np.asarray(g_gpu)
    p_gpu = np.asarray(p_gpu)
    bad_g = np.nonzero(g_gpu.view(np.uint32) != g_orc.view(np.uint32))[0]
    bad_p = np.nonzero(p_gpu != p_orc)[0]
    assert bad_g.size == 0, "%s: %d g mismatches, first %s: gpu %r oracle %r" % (
        tag, bad_g.size, bad_g[:5], g_gpu[bad_g[:5]], g_orc[bad_g[:5]])
    assert bad_p.size == 0, "%s: %d parent mismatches, first %s: gpu %r oracle %r" % (
        tag, bad_p.size, bad_p[:5], p_gpu[bad_p[:5]], p_orc[bad_p[:5]])


def assert_same_stats(tag, sg, so):
    for k in STAT_KEYS:
        assert sg[k] == so[k], "%s: %s gpu %d oracle %d" % (tag, k, sg[k], so[k])


def run_both(P, batches, plan, h_of=None, prune=True, check_insert=True, lookahead=False, truncated=False,
             timing=False):
    """Inserts `batches` into both and, after each batch i in `plan`, replans
    (root, goal) = plan[i] on both and compares everything."""
    G = gpu_graph(P)
    R = O.Graph()
    for i, b in enumerate(batches):
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
        if check_insert:
            g, p, c = G.get_policy()
            st = R.state()
            assert_same_policy("insert %d" % i, g, p, st.g, st.parent)
            assert np.array_equal(c.view(np.uint32), st.pcost.view(np.uint32))
        if i in plan:
            root, goal = plan[i]
            h = None if h_of is None else h_of(G.n)
            gg, pp, sg = G.replan(root, goal, h, prune, lookahead=lookahead, truncated=truncated, timing=timing)
            rc, so = R.replan(root, goal, h, prune, lookahead=lookahead, truncated=truncated)
            assert rc == 0 and sg["rc"] == 0
            st = R.state()
            assert_same_policy("replan %d" % i, gg, pp, st.g, st.parent)
            assert_same_stats("replan %d" % i, sg, so)
    return G, R


def test_golden_fixtures(P):
    for path in fixtures():
        fx = load_fixture(path)
        G = gpu_graph(P)
        G.insert_rows(W.from_edges(fx["n"], fx["edges"]))
        g, p, _ = G.get_policy()
        assert np.array_equal(g, fx["insert_g"]) and np.array_equal(p, fx["insert_parent"]), path
        gg, pp, st = G.replan(fx["root"], fx["goal"], fx["h"], bool(fx["prune"]))
        assert np.array_equal(gg, fx["expect_g"]), (path, gg)
        assert np.array_equal(pp, fx["expect_parent"]), (path, pp)
        for k, v in fx["expect_stats"].items():
            assert st[k] == v, (path, k, st[k], v)


@pytest.mark.parametrize("prune", [True, False])
def test_plain_2d(P, prune):
    wl = W.plain_2d()
    run_both(P, wl.batches, {0: (0, 1)}, wl.heuristic, prune)


def test_plain_2d_goal_rooted(P):
    wl = W.plain_2d()
    G, R = run_both(P, wl.batches, {0: (0, 1)}, wl.heuristic, True)
    # second Replan on the same graph, rooted at the goal, pruning off
    gg, pp, sg = G.replan(1, 0, None, False)
    rc, so = R.replan(1, 0, None, False)
    assert rc == 0
    st = R.state()
    assert_same_policy("goal-rooted", gg, pp, st.g, st.parent)
    assert_same_stats("goal-rooted", sg, so)


def test_batched_6d_small(P):
    wl = W.batched_6d(batches=12, batch=500, seed=100)
    run_both(P, wl.batches, {i: (0, 1) for i in range(12)}, wl.heuristic, True)


@pytest.mark.parametrize("d", [2, 3, 4, 8])
def test_dimensions(P, d):
    obs = W.make_obstacles(d, 20, "mixed", 40 + d)
    wl = W.grow("dim%d" % d, d, obs, 50 + d, [3000])
    run_both(P, wl.batches, {0: (0, 1)}, wl.heuristic, True)


def test_all_orphans_start(P):
    wl = W.plain_2d(samples=1500, seed=3)
    G = gpu_graph(P)
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


def test_iteration_cap(P):
    wl = W.plain_2d(samples=800, seed=4)
    G = gpu_graph(P, max_iters=2)
    R = O.Graph()
    G.insert_rows(wl.batches[0])
    R.insert_batch(wl.batches[0])
    gg, pp, sg = G.replan(0, 1, wl.heuristic(), True, allow_not_converged=True)
    rc, so = R.replan(0, 1, wl.heuristic(), True, max_iters=2)
    assert sg["rc"] == P.PIRRT_ENOTCONVERGED and rc == O.ENOTCONVERGED
    st = R.state()
    assert_same_policy("cap", gg, pp, st.g, st.parent)
    assert_same_stats("cap", sg, so)


def test_degenerate_graphs(P):
    # a lone vertex; root == goal
    G = gpu_graph(P)
    G.insert_batch(np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    g, p, st = G.replan(0, 0)
    assert g[0] == 0 and p[0] == -1 and st["iterations"] == 1
    # empty batch is a no-op
    G.insert_batch(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert G.n == 1
    # isolated vertices, a detached component and zero-cost edges
    edges = [(0, 2, 0.0), (2, 3, 1.0), (4, 5, 1.0), (5, 6, 0.5), (3, 1, 2.0)]
    b = W.from_edges(8, edges)
    G2 = gpu_graph(P)
    R = O.Graph()
    G2.insert_rows(b)
    R.insert_batch(b)
    for prune in (True, False):
        gg, pp, sg = G2.replan(0, 1, None, prune)
        rc, so = R.replan(0, 1, None, prune)
        st = R.state()
        assert_same_policy("degenerate", gg, pp, st.g, st.parent)
        assert_same_stats("degenerate", sg, so)
    assert np.isinf(gg[4:]).all() and gg[7] == np.inf


def test_permuted_row_order_is_invisible(P):
    """The entries of every input row shuffled: insertion and Replan take lexicographic
    minima, so the policy, g and counters are the same bits as for the rows in order
    (and as the oracle's)."""
    import dataclasses
    wl = W.plain_2d(samples=3000, seed=12)
    b = wl.batches[0]
    rng = np.random.default_rng(5)
    col, cost = b.col.copy(), b.cost.copy()
    for v in range(b.n_new):
        a, e = int(b.row_ptr[v]), int(b.row_ptr[v + 1])
        perm = a + rng.permutation(e - a)
        col[a:e], cost[a:e] = b.col[perm], b.cost[perm]
    bp = dataclasses.replace(b, col=col, cost=cost)
    h = wl.heuristic(wl.n)
    outs = []
    for batch in (b, bp):
        G = gpu_graph(P)
        G.insert_rows(batch)
        gi, pi, _ = G.get_policy()
        gg, pp, sg = G.replan(0, 1, h, True)
        outs.append((np.asarray(gi).copy(), np.asarray(pi).copy(), np.asarray(gg).copy(), np.asarray(pp).copy(), sg))
    R = O.Graph()
    assert R.insert_batch(bp) == 0
    rc, so = R.replan(0, 1, h, True)
    st = R.state()
    for tag, (gi, pi, gg, pp, sg) in zip(("rows in order", "rows shuffled"), outs):
        assert_same_policy(tag, gg, pp, st.g, st.parent)
        assert_same_stats(tag, sg, so)
    assert np.array_equal(outs[0][0].view(np.uint32), outs[1][0].view(np.uint32))
    assert np.array_equal(outs[0][1], outs[1][1])


def test_rows_longer_than_a_wave(P):
    # a hub with 300 neighbours and a ring: rows far longer than 64 entries
    rng = np.random.default_rng(9)
    n = 400
    edges = [(0, v, float(np.float32(rng.uniform(0.5, 2.0)))) for v in range(2, 302)]
    edges += [(v, v + 1, float(np.float32(rng.uniform(0.1, 0.3)))) for v in range(1, n - 1)]
    edges += [(1, n - 1, 0.25)]
    b = W.from_edges(n, edges)
    run_both(P, [b], {0: (0, 1)}, None, False)
    run_both(P, [b], {0: (5, 1)}, None, True)


def test_device_buffers(P):
    import torch
    wl = W.plain_2d(samples=1200, seed=6)
    b = wl.batches[0]
    dev = torch.device("cuda:0")
    G = gpu_graph(P)
    G.insert_batch(torch.from_numpy(b.row_ptr).to(dev), torch.from_numpy(b.col).to(dev),
                   torch.from_numpy(b.cost).to(dev))
    h = torch.from_numpy(wl.heuristic()).to(dev)
    gg, pp, sg = G.replan(0, 1, h, True)
    assert gg.is_cuda and pp.is_cuda
    R = O.Graph()
    R.insert_batch(b)
    rc, so = R.replan(0, 1, wl.heuristic(), True)
    st = R.state()
    assert_same_policy("device", gg.cpu().numpy(), pp.cpu().numpy(), st.g, st.parent)
    assert_same_stats("device", sg, so)


def test_invalid_arguments_leave_state(P):
    wl = W.plain_2d(samples=300, seed=7)
    G = gpu_graph(P)
    G.insert_rows(wl.batches[0])
    n0, e0 = G.n, G.nnz
    before = G.get_policy()
    bad = [
        (np.array([0, 1], np.int64), np.array([n0], np.int32), np.array([1.0], np.float32)),   # col == own id
        (np.array([0, 1], np.int64), np.array([-1], np.int32), np.array([1.0], np.float32)),   # negative col
        (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([np.nan], np.float32)),  # NaN cost
        (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([-0.0], np.float32)),   # -0.0 cost
        (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([np.inf], np.float32)),  # inf cost
        (np.array([1, 1], np.int64), np.array([0], np.int32), np.array([1.0], np.float32)),    # row_ptr[0] != 0
    ]
    for rp, c, w in bad:
        with pytest.raises(P.PirrtError) as e:
            G.insert_batch(rp, c, w)
        assert e.value.code == P.PIRRT_EINVAL
    assert G.n == n0 and G.nnz == e0
    after = G.get_policy()
    for x, y in zip(before, after):
        assert np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32))
    for root, goal in ((-1, 1), (0, n0), (n0, 0)):
        with pytest.raises(P.PirrtError) as e:
            G.replan(root, goal)
        assert e.value.code == P.PIRRT_EINVAL
    h = wl.heuristic()
    h[3] = np.nan
    with pytest.raises(P.PirrtError):
        G.replan(0, 1, h)
    h[3] = -1.0
    with pytest.raises(P.PirrtError):
        G.replan(0, 1, h)


def test_device_allocation_failure(P):
    """An adjacency reservation far beyond the device's memory (2^42 entries): creation
    reports ENOMEM without a handle, and the device stays usable for the next graph."""
    with pytest.raises(P.PirrtError) as e:
        gpu_graph(P, edge_capacity=1 << 42)
    assert e.value.code == P.PIRRT_ENOMEM
    wl = W.plain_2d(samples=500, seed=13)
    run_both(P, wl.batches, {0: (0, 1)}, wl.heuristic, True)


def test_injected_launch_failure_poisons_the_handle(P, monkeypatch):
    """A HIP error in a Replan (forced on the host by PIRRT_FAULT_INJECT=launch; no
    kernel faults) returns EDEVICE, and every later call on that handle returns
    EDEVICE too; destroying it works, and another handle on the device is unaffected."""
    wl = W.plain_2d(samples=2000, seed=14)
    monkeypatch.setenv("PIRRT_FAULT_INJECT", "launch")
    G = gpu_graph(P)
    monkeypatch.delenv("PIRRT_FAULT_INJECT")
    G.insert_rows(wl.batches[0])
    with pytest.raises(P.PirrtError) as e:
        G.replan(0, 1, wl.heuristic(), True)
    assert e.value.code == P.PIRRT_EDEVICE
    assert "injected" in str(e.value)
    for call in (lambda: G.replan(0, 1, wl.heuristic(), True), lambda: G.get_policy(),
                 lambda: G.insert_rows(wl.batches[0]), lambda: G.snapshot_save()):
        with pytest.raises(P.PirrtError) as e:
            call()
        assert e.value.code == P.PIRRT_EDEVICE
    G.close()
    run_both(P, wl.batches, {0: (0, 1)}, wl.heuristic, True)


def test_injected_allocation_failure_leaves_the_graph_unchanged(P, monkeypatch):
    """A failed growth of the vertex storage (forced on the host by
    PIRRT_FAULT_INJECT=alloc) returns ENOMEM with the graph as it was; the same
    insertion then succeeds and the results equal the oracle's."""
    wl = W.batched_6d(batches=2, batch=1500, seed=105)
    monkeypatch.setenv("PIRRT_FAULT_INJECT", "alloc")
    G = gpu_graph(P)
    monkeypatch.delenv("PIRRT_FAULT_INJECT")
    R = O.Graph()
    b0, b1 = wl.batches
    with pytest.raises(P.PirrtError) as e:
        G.insert_rows(b0)
    assert e.value.code == P.PIRRT_ENOMEM and G.n == 0
    for b in (b0, b1):
        G.insert_rows(b)
        assert R.insert_batch(b) == 0
    gg, pp, sg = G.replan(0, 1, wl.heuristic(G.n), True)
    rc, so = R.replan(0, 1, wl.heuristic(G.n), True)
    st = R.state()
    assert_same_policy("after ENOMEM", gg, pp, st.g, st.parent)
    assert_same_stats("after ENOMEM", sg, so)


def test_snapshot_restore_repeatable(P):
    wl = W.batched_6d(batches=2, batch=2000, seed=100)
    G = gpu_graph(P)
    for b in wl.batches:
        G.insert_rows(b)
    G.snapshot_save()
    outs = []
    for _ in range(3):
        G.snapshot_restore()
        g, p, st = G.replan(0, 1, wl.heuristic(), True)
        outs.append((g.copy(), p.copy(), st))
    for g, p, st in outs[1:]:
        assert np.array_equal(g.view(np.uint32), outs[0][0].view(np.uint32))
        assert np.array_equal(p, outs[0][1])
        assert_same_stats("repeat", st, outs[0][2])


def test_adjacency_is_symmetric_union(P):
    wl = W.batched_6d(batches=3, batch=700, seed=101)
    G = gpu_graph(P)
    R = O.Graph()
    for b in wl.batches:
        G.insert_rows(b)
        R.insert_batch(b)
    pg, ng, cg = G.adjacency()
    po, no, co = R.adjacency()
    assert np.array_equal(pg, po)
    for v in range(G.n):
        a = sorted(zip(ng[pg[v]:pg[v + 1]].tolist(), cg[pg[v]:pg[v + 1]].view(np.uint32).tolist()))
        b = sorted(zip(no[po[v]:po[v + 1]].tolist(), co[po[v]:po[v + 1]].view(np.uint32).tolist()))
        assert a == b, v


def lattice_batch(side, keep_frac, seed, shuffle=True):
    rng = np.random.default_rng(seed)
    keep = rng.random((side, side)) < keep_frac
    keep[0, 0] = keep[side - 1, side - 1] = True
    cells = [(i, j) for i in range(side) for j in range(side) if keep[i, j]]
    start, end = cells.index((0, 0)), cells.index((side - 1, side - 1))
    rest = [k for k in range(len(cells)) if k not in (start, end)]
    if shuffle:
        rest = list(rng.permutation(rest))
    order = [start, end] + rest
    label = {cells[k]: i for i, k in enumerate(order)}
    edges = []
    for (i, j) in cells:
        for (a, b) in ((i + 1, j), (i, j + 1), (i + 1, j + 1)):
            if (a, b) in label:
                edges.append((label[(i, j)], label[(a, b)], 1.0 if a == i or b == j else 1.5))
    return W.from_edges(len(cells), edges)


@pytest.mark.parametrize("prune", [True, False])
def test_lattice_ties(P, prune):
    """Unit-cost lattice with diagonals: equal candidates everywhere, so every
    minimum is decided by the neighbour id (and storage renumbering must not leak)."""
    b = lattice_batch(60, 0.85, 12)
    run_both(P, [b], {0: (0, 1)}, None, prune)


def test_renumbering_is_invisible(P, monkeypatch):
    wl = W.batched_6d(batches=5, batch=800, seed=102)
    outs = []
    monkeypatch.setenv("PIRRT_REORDER_MIN", "0")  # renumber small graphs too
    for growth in ("0", "1.0", "1.25"):
        monkeypatch.setenv("PIRRT_REORDER_GROWTH", growth)
        G = gpu_graph(P)
        res = []
        for b in wl.batches:
            G.insert_rows(b)
            g, p, st = G.replan(0, 1, wl.heuristic(G.n), True)
            res.append((g.copy(), p.copy(), {k: st[k] for k in STAT_KEYS}))
        outs.append(res)
    for other in outs[1:]:
        for (g0, p0, s0), (g1, p1, s1) in zip(outs[0], other):
            assert np.array_equal(g0.view(np.uint32), g1.view(np.uint32))
            assert np.array_equal(p0, p1)
            assert s0 == s1


def test_level_synchronous_evaluator_agrees(P, monkeypatch):
    """The two GPU evaluators (walk with stamps, level-synchronous BFS) must give
    the oracle's results bit for bit."""
    monkeypatch.setenv("PIRRT_EVALUATE", "levels")
    wl = W.batched_6d(batches=4, batch=1500, seed=103)
    run_both(P, wl.batches, {i: (0, 1) for i in range(4)}, wl.heuristic, True)
    b = lattice_batch(40, 0.9, 5)
    run_both(P, [b], {0: (0, 1)}, None, False)


@pytest.mark.parametrize("evaluator", ["levels", "walk"])
def test_repeated_replans_with_a_new_root(P, monkeypatch, evaluator):
    """Repeated Replans on one graph replay captured loop bodies; a later Replan with
    another root on the same graph (and the same arguments otherwise) must not replay
    anything tied to the old root.  Root 0 twice, then root k twice, then root 0
    again, each against the oracle from the same state."""
    monkeypatch.setenv("PIRRT_EVALUATE", evaluator)
    wl = W.batched_6d(batches=1, batch=3000, seed=104)
    G = gpu_graph(P)
    R = O.Graph()
    b = wl.batches[0]
    G.insert_rows(b)
    assert R.insert_batch(b) == 0
    n = G.n
    h = wl.heuristic(n)
    k = n // 2
    for call, (root, goal) in enumerate([(0, 1), (0, 1), (k, 1), (k, 1), (0, 1)]):
        gg, pp, sg = G.replan(root, goal, h, True)
        rc, so = R.replan(root, goal, h, True)
        assert rc == 0
        st = R.state()
        assert_same_policy("%s call %d root %d" % (evaluator, call, root), gg, pp, st.g, st.parent)
        assert_same_stats("%s call %d root %d" % (evaluator, call, root), sg, so)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("coherent", [0, 1])
def test_every_kernel_configuration(P, monkeypatch, variant, coherent):
    """The autotuner may choose any row split and stamp scope: each gives the
    oracle's results."""
    monkeypatch.setenv("PIRRT_ROW_VARIANT", str(variant))
    monkeypatch.setenv("PIRRT_WALK_COHERENT", str(coherent))
    wl = W.batched_6d(batches=3, batch=800, seed=101)
    run_both(P, wl.batches, {0: (0, 1), 2: (0, 1)}, wl.heuristic, True, check_insert=False)


@pytest.mark.parametrize("parts", [2, 3])
def test_walk_in_parts(P, monkeypatch, parts):
    """The walk split over consecutive slot ranges (one launch each; the first also takes
    the finish step after an Improve) gives the oracle's results and counters."""
    monkeypatch.setenv("PIRRT_WALK_PARTS", str(parts))
    wl = W.batched_6d(batches=3, batch=800, seed=103)
    run_both(P, wl.batches, {0: (0, 1), 1: (5, 1), 2: (0, 1)}, wl.heuristic, True, check_insert=False)


def test_tune_restores_policy_and_keeps_results(P):
    wl = W.plain_2d()
    G = gpu_graph(P)
    G.insert_rows(wl.batches[0])
    g0, p0, c0 = G.get_policy()
    h = wl.heuristic(G.n)
    cfg = G.tune(0, 1, h, True)
    assert 0 <= cfg < 8
    g1, p1, c1 = G.get_policy()
    assert np.array_equal(g0.view(np.uint32), g1.view(np.uint32)) and np.array_equal(p0, p1)
    assert np.array_equal(c0.view(np.uint32), c1.view(np.uint32))
    R = O.Graph()
    assert R.insert_batch(wl.batches[0]) == 0
    gg, pp, sg = G.replan(0, 1, h, True)
    rc, so = R.replan(0, 1, h, True)
    st = R.state()
    assert_same_policy("after tune", gg, pp, st.g, st.parent)
    assert_same_stats("after tune", sg, so)


def test_breadth_first_order_agrees(P, monkeypatch):
    """Both storage orders (clustered, plain breadth-first) give the oracle's results."""
    monkeypatch.setenv("PIRRT_ORDER", "bfs")
    wl = W.batched_6d(batches=4, batch=700, seed=103)
    run_both(P, wl.batches, {i: (0, 1) for i in range(4)}, wl.heuristic, True)


# ---- narrowed Improve domain (PIRRT_LOOKAHEAD) against the oracle's mode of it

@pytest.mark.parametrize("case", ["2d", "6d_batches", "6d_30k", "8d"])
def test_lookahead_domain(P, case):
    if case == "2d":
        wl = W.plain_2d()
        plan = {0: (0, 1)}
    elif case == "6d_batches":
        wl = W.batched_6d(batches=4, batch=700, seed=103)
        plan = {i: (0, 1) for i in range(4)}
    elif case == "6d_30k":
        wl = W.plain_6d(samples=30_000, extra=2_000, seed=205)
        plan = {0: (0, 1), 1: (0, 1)}
    else:
        wl = W.grow("8d", 8, W.make_obstacles(8, 20, "sphere", 7), 8, [3000, 1000])
        plan = {0: (0, 1), 1: (0, 1)}
    run_both(P, wl.batches, plan, wl.heuristic, True, check_insert=False, lookahead=True)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_lookahead_every_row_split(P, monkeypatch, variant):
    monkeypatch.setenv("PIRRT_ROW_VARIANT", str(variant))
    wl = W.batched_6d(batches=3, batch=800, seed=104)
    run_both(P, wl.batches, {0: (0, 1), 2: (0, 1)}, wl.heuristic, True, check_insert=False, lookahead=True)


def test_lookahead_without_pruning_is_the_full_domain(P):
    wl = W.batched_6d(batches=2, batch=900, seed=106)
    G = gpu_graph(P)
    for b in wl.batches:
        G.insert_rows(b)
    G.snapshot_save()
    h = wl.heuristic(G.n)
    g1, p1, s1 = G.replan(0, 1, h, False, lookahead=True)
    G.snapshot_restore()
    g2, p2, s2 = G.replan(0, 1, h, False, lookahead=False)
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32)) and np.array_equal(p1, p2)
    assert_same_stats("lookahead without pruning", s1, s2)


def test_lookahead_worked_example(P):
    """The hand-worked five-vertex example of the oracle pins, on the device."""
    from oracle_pins import lookahead_example
    edges, h, parent, pcost = lookahead_example()
    want = {False: (2, 5, 8, 16, 1), True: (2, 5, 4, 10, 1)}
    for look in (False, True):
        G = gpu_graph(P)
        G.insert_rows(W.from_edges(5, edges))
        G.set_policy(np.zeros(5, np.float32), parent, pcost)
        g, p, st = G.replan(0, 1, h, True, lookahead=look)
        got = (st["iterations"], st["sum_P"], st["sum_D"], st["edges_examined"], st["changed_total"])
        assert got == want[look], (look, got)
        assert np.array_equal(g, np.array([0, 2, 1, 0.5, 1.5], np.float32))
        assert np.array_equal(p, np.array([-1, 2, 0, 0, 2], np.int32))


# ---- truncated Evaluate (PIRRT_TRUNCATED) against the oracle's mode of it

@pytest.mark.parametrize("case", ["2d", "2d_noprune", "6d_batches", "6d_30k", "2d_1200"])
def test_truncated_evaluate(P, case):
    """Every Replan of the plan in the truncated mode; the next batch is inserted on top
    of the stale g it leaves, and the insertion-time policy is compared too."""
    prune = case != "2d_noprune"
    if case in ("2d", "2d_noprune"):
        wl = W.plain_2d()
        plan = {0: (0, 1)}
    elif case == "6d_batches":
        wl = W.batched_6d(batches=4, batch=700, seed=103)
        plan = {i: (0, 1) for i in range(4)}
    elif case == "6d_30k":
        wl = W.plain_6d(samples=30_000, extra=2_000, seed=205)
        plan = {0: (0, 1), 1: (0, 1)}
    else:  # small enough for the single-workgroup path, which the truncated mode skips
        wl = W.plain_2d(samples=1200, seed=8)
        plan = {0: (0, 1)}
    run_both(P, wl.batches, plan, wl.heuristic, prune, check_insert=True, truncated=True)


@pytest.mark.parametrize("variant,coherent", [(v, c) for v in range(4) for c in ("0", "1")])
def test_truncated_every_configuration(P, monkeypatch, variant, coherent):
    monkeypatch.setenv("PIRRT_ROW_VARIANT", str(variant))
    monkeypatch.setenv("PIRRT_WALK_COHERENT", coherent)
    wl = W.batched_6d(batches=3, batch=600, seed=108)
    run_both(P, wl.batches, {0: (0, 1), 2: (0, 1)}, wl.heuristic, True, check_insert=False, truncated=True)


def test_truncated_direct_launches_and_level_setting(P, monkeypatch):
    """The timing pass (direct launches), and PIRRT_EVALUATE=levels, which the truncated
    mode overrides with its walk."""
    wl = W.batched_6d(batches=2, batch=800, seed=109)
    run_both(P, wl.batches, {0: (0, 1), 1: (0, 1)}, wl.heuristic, True, check_insert=False, truncated=True,
             timing=True)
    monkeypatch.setenv("PIRRT_EVALUATE", "levels")
    run_both(P, wl.batches, {1: (0, 1)}, wl.heuristic, True, check_insert=False, truncated=True)


def test_truncated_worked_example(P):
    """The hand-worked six-vertex example of the oracle pins, on the device: vertex 4
    is skipped by the walks and keeps g = 7 although its path costs 6."""
    from oracle_pins import truncated_example
    edges, g0, parent, pcost = truncated_example()
    want = {True: ((2, 4, 6, 14, 1), [0, 4, 2, 5, 7, 1]), False: ((2, 6, 8, 16, 1), [0, 4, 2, 5, 6, 1])}
    for trunc in (True, False):
        G = gpu_graph(P)
        G.insert_rows(W.from_edges(6, edges))
        G.set_policy(g0, parent, pcost)
        g, p, st = G.replan(0, 1, np.zeros(6, np.float32), True, truncated=trunc)
        got = (st["iterations"], st["sum_P"], st["sum_D"], st["edges_examined"], st["changed_total"])
        assert got == want[trunc][0], (trunc, got)
        assert np.array_equal(g, np.array(want[trunc][1], np.float32)), (trunc, g)
        assert np.array_equal(p, np.array([-1, 0, 5, 2, 3, 0], np.int32))


def test_truncated_after_other_root_and_rejections(P):
    """A truncated Replan rooted at the goal after one rooted at x_init reads the stale
    g(goal) of the first as its threshold, as the oracle does; the mode is refused
    together with PIRRT_LOOKAHEAD and for batches, leaving the state as it was."""
    wl = W.plain_2d(samples=3000, seed=9)
    G = gpu_graph(P)
    R = O.Graph()
    G.insert_rows(wl.batches[0])
    assert R.insert_batch(wl.batches[0]) == 0
    h = wl.heuristic(G.n)
    for root, goal in ((0, 1), (1, 0), (0, 1)):
        gg, pp, sg = G.replan(root, goal, h, True, truncated=True)
        rc, so = R.replan(root, goal, h, True, truncated=True)
        assert rc == 0
        st = R.state()
        assert_same_policy("root %d" % root, gg, pp, st.g, st.parent)
        assert_same_stats("root %d" % root, sg, so)
    before = G.get_policy()
    with pytest.raises(P.PirrtError):
        G.replan(0, 1, h, True, truncated=True, lookahead=True)
    after = G.get_policy()
    assert all(np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32))
               for a, b in zip(before, after))
    B = P.Batch()
    b0 = wl.batches[0]
    B.add_problem(b0.row_ptr, b0.col, b0.cost)
    roots = np.zeros(1, np.int32)
    goals = np.ones(1, np.int32)
    rc = B._lib.pirrt_batch_replan(B._h, roots.ctypes.data, goals.ctypes.data, None, P.PIRRT_TRUNCATED, None,
                                   None, P.PIRRT_MEM_HOST, None)
    assert rc == P.PIRRT_EINVAL


def test_truncated_degenerate_graphs(P):
    """The truncated mode on a lone vertex (root == goal), on isolated vertices, a
    detached component and zero-cost edges, and from a policy whose parents form a
    cycle (the walk must leave the cycle's vertices unvisited, with their old g, until
    Improve breaks it); both modes, pruning on and off, against the oracle."""
    G = gpu_graph(P)
    G.insert_batch(np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    g, p, st = G.replan(0, 0, truncated=True)
    assert g[0] == 0 and p[0] == -1 and st["iterations"] == 1 and st["sum_P"] == 0
    b = W.from_edges(8, [(0, 2, 0.0), (2, 3, 1.0), (4, 5, 1.0), (5, 6, 0.5), (3, 1, 2.0)])
    for prune in (True, False):
        G2 = gpu_graph(P)
        R = O.Graph()
        G2.insert_rows(b)
        R.insert_batch(b)
        gg, pp, sg = G2.replan(0, 1, None, prune, truncated=True)
        rc, so = R.replan(0, 1, None, prune, truncated=True)
        assert rc == 0
        st = R.state()
        assert_same_policy("degenerate truncated", gg, pp, st.g, st.parent)
        assert_same_stats("degenerate truncated", sg, so)
    cyc = W.from_edges(5, [(0, 1, 1.0), (1, 2, 1.0), (2, 3, 1.0), (3, 4, 1.0), (0, 4, 5.0)])
    g0 = np.array([0, 1, 7, 8, 9], np.float32)
    par = np.array([-1, 0, 3, 2, 3], np.int32)
    pc = np.array([0, 1, 1, 1, 1], np.float32)
    for trunc in (True, False):
        for prune in (True, False):
            G3 = gpu_graph(P)
            R = O.Graph()
            G3.insert_rows(cyc)
            R.insert_batch(cyc)
            G3.set_policy(g0, par, pc)
            assert R.set_state(g0, par, pc) == 0
            gg, pp, sg = G3.replan(0, 4, None, prune, truncated=trunc)
            rc, so = R.replan(0, 4, None, prune, truncated=trunc)
            assert rc == 0
            st = R.state()
            tag = "cycle truncated=%s prune=%s" % (trunc, prune)
            assert_same_policy(tag, gg, pp, st.g, st.parent)
            assert_same_stats(tag, sg, so)
            assert np.array_equal(pp, np.array([-1, 0, 1, 2, 3], np.int32)), (tag, pp)


@pytest.mark.parametrize("prune,lookahead", [(True, False), (False, False), (True, True)])
def test_single_workgroup_path_agrees(P, monkeypatch, prune, lookahead):
    """Graphs of up to 1,536 vertices take the single-workgroup Replan; the multi-kernel
    loop (PIRRT_SMALL=0) and the oracle must give the same policy and counters."""
    cases = [W.plain_2d(samples=1530, seed=3), W.batched_6d(batches=2, batch=700, seed=107),
             W.plain_2d(samples=60, seed=5), W.plain_2d(samples=1534, seed=6)]
    for wl in cases:
        outs = []
        for small in ("1", "0"):
            monkeypatch.setenv("PIRRT_SMALL", small)
            G = gpu_graph(P)
            for b in wl.batches:
                G.insert_rows(b)
            h = wl.heuristic(G.n)
            g, p, st = G.replan(0, 1, h, prune, lookahead=lookahead)
            outs.append((np.asarray(g).copy(), np.asarray(p).copy(), st))
        R = O.Graph()
        for b in wl.batches:
            assert R.insert_batch(b) == 0
        rc, so = R.replan(0, 1, wl.heuristic(R.n), prune, lookahead=lookahead)
        st_o = R.state()
        for tag, (g, p, st) in zip(("single workgroup", "multi-kernel"), outs):
            assert_same_policy("%s %s" % (wl.name, tag), g, p, st_o.g, st_o.parent)
            assert_same_stats("%s %s" % (wl.name, tag), st, so)


def test_single_workgroup_iteration_cap(P):
    """The cap inside the single-workgroup loop: ENOTCONVERGED after exactly the capped
    passes, with the oracle's policy at that point."""
    wl = W.plain_2d(samples=1500, seed=4)
    for cap in (1, 2, 3):
        G = gpu_graph(P, max_iters=cap)
        G.insert_rows(wl.batches[0])
        h = wl.heuristic(G.n)
        g, p, st = G.replan(0, 1, h, True, allow_not_converged=True)
        R = O.Graph()
        assert R.insert_batch(wl.batches[0]) == 0
        rc, so = R.replan(0, 1, h, True, max_iters=cap)
        assert rc == O.ENOTCONVERGED and st["rc"] == P.PIRRT_ENOTCONVERGED
        fin = R.state()
        assert_same_policy("cap %d" % cap, g, p, fin.g, fin.parent)
        assert_same_stats("cap %d" % cap, st, so)
