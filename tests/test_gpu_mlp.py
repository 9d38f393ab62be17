"""The learned proposal's network on the device (pirrt_mlp_* through the C ABI)
against the oracle (oracle/mlp.py).

Tolerance, from the arithmetic: both sides use the same bfloat16 inputs and weights
and exact products; only the accumulation differs (binary32 on the device, binary64
in the oracle).  An activation can therefore differ by one bfloat16 ulp (2^-8
relative) where the two sums fall on opposite sides of a rounding boundary, and such a
difference moves the logit by at most 2^-8 times the absolute path sum downstream of
it.  The bound used is twice that sum over every activation (accumulation error
included), per logit; the median error must also be far below it, so a systematic
mistake (a wrong lane layout, a dropped bias) cannot hide under the bound.
Gradients are compared element by element against bounds derived the same way
(gradient_bounds), and Adam against the oracle's Adam."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu

IN_DIM = 286


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_04920_amd as P
    P.load()
    return P


def flat(p: M.Params) -> np.ndarray:
    return np.concatenate([np.asarray(getattr(p, k), np.float32).ravel() for k in M.PARAM_NAMES])


def unflat(v: np.ndarray) -> dict:
    out, o = {}, 0
    shapes = {"W1": (M.K_IN, M.HIDDEN), "b1": (M.HIDDEN,), "W2": (M.HIDDEN, M.HIDDEN), "b2": (M.HIDDEN,),
              "w3": (M.HIDDEN,), "b3": (1,)}
    for k in M.PARAM_NAMES:
        n = int(np.prod(shapes[k]))
        out[k] = v[o:o + n].reshape(shapes[k])
        o += n
    return out


def problem(seed, B):
    rng = np.random.default_rng(seed)
    p = M.init_params(rng, IN_DIM)
    p.b1[:] = (rng.standard_normal(M.HIDDEN) * 0.1).astype(np.float32)
    p.b2[:] = (rng.standard_normal(M.HIDDEN) * 0.1).astype(np.float32)
    p.b3[:] = 0.2
    x = rng.random((B, IN_DIM)).astype(np.float32)
    y = (rng.random(B) < 0.4).astype(np.float32)
    return p, x, y


def logit_bound(p, x):
    _, (X, Z1, A1, Z2, A2) = M.forward(p, x)
    aw3 = np.abs(M.bf16(p.w3))
    down1 = np.abs(M.bf16(p.W2)) @ aw3
    return 2.0 * 2.0 ** -8 * (np.abs(A2) @ aw3 + np.abs(A1) @ down1) + 1e-6


@pytest.mark.parametrize("B", [1, 100, 256, 1000])
def test_forward(P, B):
    p, x, _ = problem(10 + B, B)
    net = P.Mlp(IN_DIM, 1024)
    assert net.num_params == flat(p).size
    net.set_params(flat(p))
    assert np.array_equal(net.get_params(), flat(p))
    z = net.forward(x)
    want, _ = M.forward(p, x)
    err = np.abs(z - want)
    bound = logit_bound(p, x)
    assert np.all(err <= bound), (np.max(err / bound), B)
    assert np.median(err) <= 1e-3 * np.median(bound) + 1e-6


def test_forward_device_buffers(P):
    import torch
    p, x, _ = problem(3, 300)
    net = P.Mlp(IN_DIM, 512, stream=torch.cuda.current_stream().cuda_stream)
    net.set_params(torch.from_numpy(flat(p)).cuda())
    z = net.forward(torch.from_numpy(x).cuda())
    assert z.is_cuda
    want, _ = M.forward(p, x)
    assert np.all(np.abs(z.cpu().numpy() - want) <= logit_bound(p, x))


U = 2.0 ** -24  # unit roundoff of binary32
C_ACC = 2.0  # slack on the binary32 accumulation bound (k - 1) u (matrix-core sums)


def _spread(o, lo, hi, zero):
    """Largest distance from the oracle's bfloat16 value o to bf16 of any value in
    [lo, hi] (and to 0 where `zero`: a ReLU mask the device may decide the other
    way).  bf16 rounding is monotone, so the interval's ends bound it."""
    d = np.maximum(np.abs(M.bf16(lo) - o), np.abs(M.bf16(hi) - o))
    return np.where(zero, np.maximum(d, np.abs(o)), d)


def gradient_bounds(p, x, y, exact_forward=False):
    """Per-element bounds on |device - oracle| for the loss gradient.

    Both sides take the same bfloat16 operands; the device sums in binary32 and
    the oracle in binary64.  A binary32 sum of k terms is within (k - 1) u of the
    exact sum of |terms| (u = 2^-24); the slack C_ACC covers the matrix cores'
    grouping of partial sums.  Every rounding to bfloat16 (activations, dZ2, dZ1)
    is bounded by where it can land over the interval of pre-rounding values the
    device may hold (usually the oracle's own value: then the bound is 0), and a
    ReLU mask whose argument lies within its error bound of 0 may go either way.
    The error intervals are carried through every product with absolute values
    (first order: products of two errors are added too), forward to the logit and
    backward to each gradient element.  exact_forward: the caller has checked that
    both hidden layers' sums are exact in binary32 (quantized_problem), so the two
    sides' Z1, A1, Z2, A2 and ReLU masks are identical."""
    f64 = np.float64
    B = len(y)
    y = np.asarray(y, f64)
    z, (X, Z1, A1, Z2, A2) = M.forward(p, x)
    W1b, W2b, w3b = M.bf16(p.W1), M.bf16(p.W2), M.bf16(p.w3)
    aW1, aW2, aw3 = np.abs(W1b), np.abs(W2b), np.abs(w3b)
    gam = lambda k: C_ACC * k * U  # noqa: E731
    # forward
    eZ1 = gam(M.K_IN + 1) * (np.abs(X) @ aW1 + np.abs(p.b1.astype(f64)))
    if exact_forward:
        eZ1 = np.zeros_like(Z1)
    dA1 = _spread(A1, np.maximum(Z1 - eZ1, 0), np.maximum(Z1 + eZ1, 0), False)
    eZ2 = dA1 @ aW2 + gam(M.HIDDEN + 1) * ((np.abs(A1) + dA1) @ aW2 + np.abs(p.b2.astype(f64)))
    if exact_forward:
        eZ2 = np.zeros_like(Z2)
    dA2 = _spread(A2, np.maximum(Z2 - eZ2, 0), np.maximum(Z2 + eZ2, 0), False)
    ez = dA2 @ aw3 + gam(M.HIDDEN + 1) * ((np.abs(A2) + dA2) @ aw3 + abs(float(p.b3[0])))
    # backward
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    edz = ez / (4.0 * B) + 4.0 * U / B + 4.0 * U * np.abs(dz)
    bounds = {}
    bounds["w3"] = dA2.T @ np.abs(dz) + (np.abs(A2) + dA2).T @ edz + \
        gam(B) * ((np.abs(A2) + dA2).T @ (np.abs(dz) + edz))
    bounds["b3"] = np.array([edz.sum() + gam(B) * (np.abs(dz) + edz).sum()])
    pre2 = np.outer(dz, w3b)
    e2 = np.outer(edz, aw3) + U * np.abs(pre2)
    mask2 = (Z2 > 0).astype(f64)
    dZ2 = M.bf16(pre2 * mask2)
    amb2 = np.abs(Z2) <= eZ2
    lo2 = np.where(mask2 > 0, pre2 - e2, 0.0)
    hi2 = np.where(mask2 > 0, pre2 + e2, 0.0)
    lo2 = np.where(amb2, pre2 - e2, lo2)
    hi2 = np.where(amb2, pre2 + e2, hi2)
    ddZ2 = _spread(dZ2, lo2, hi2, amb2)
    aA1, adZ2 = np.abs(A1) + dA1, np.abs(dZ2) + ddZ2
    bounds["W2"] = dA1.T @ np.abs(dZ2) + aA1.T @ ddZ2 + gam(B) * (aA1.T @ adZ2)
    bounds["b2"] = ddZ2.sum(axis=0) + gam(B) * adZ2.sum(axis=0)
    pre1 = dZ2 @ W2b.T
    e1 = ddZ2 @ aW2.T + gam(M.HIDDEN) * (adZ2 @ aW2.T)
    mask1 = (Z1 > 0).astype(f64)
    dZ1 = M.bf16(pre1 * mask1)
    amb1 = np.abs(Z1) <= eZ1
    lo1 = np.where(mask1 > 0, pre1 - e1, 0.0)
    hi1 = np.where(mask1 > 0, pre1 + e1, 0.0)
    lo1 = np.where(amb1, pre1 - e1, lo1)
    hi1 = np.where(amb1, pre1 + e1, hi1)
    ddZ1 = _spread(dZ1, lo1, hi1, amb1)
    adZ1 = np.abs(dZ1) + ddZ1
    bounds["W1"] = np.abs(X).T @ ddZ1 + gam(B) * (np.abs(X).T @ adZ1)
    bounds["b1"] = ddZ1.sum(axis=0) + gam(B) * adZ1.sum(axis=0)
    return bounds


@pytest.mark.parametrize("B", [64, 200, 512])
def test_gradients(P, B):
    """Every gradient element within its bound (gradient_bounds), and the typical
    error far below the bound, so a wrong element, a dropped batch row or a wrong
    tile cannot hide."""
    p, x, y = problem(20 + B, B)
    net = P.Mlp(IN_DIM, 512)
    net.set_params(flat(p))
    loss, g = net.gradients(x, y)
    want_loss, want, _ = M.loss_and_grads(p, x, y)
    assert abs(loss - want_loss) <= 1e-3 * abs(want_loss) + 1e-5
    gd = unflat(g)
    bounds = gradient_bounds(p, x, y)
    for k in M.PARAM_NAMES:
        ref = np.asarray(want[k], np.float64).reshape(gd[k].shape)
        bnd = 2.0 * bounds[k].reshape(gd[k].shape)
        err = np.abs(gd[k].astype(np.float64) - ref)
        over = np.nonzero(err > bnd)
        assert over[0].size == 0, (k, over[0][:5], err[over][:5], bnd[over][:5])
        live = bnd > 0
        if live.sum() > 16:
            assert np.median(err[live] / bnd[live]) < 0.05, (k, np.median(err[live] / bnd[live]))
    assert np.all(gd["W1"][IN_DIM:] == 0.0)  # padding rows of X are zero


def quantized_problem(seed, B):
    """Inputs on a grid that makes both hidden layers exact in binary32: features
    k/16, W1 and W2 on multiples of 2^-6 (|W1| <= 12/64, |W2| <= 4/64), b1 on
    2^-10, b2 on 2^-16.  Every product of the first layer is then a multiple of
    2^-10 and every A1 a multiple of 2^-10 (bfloat16 of a multiple of 2^-10 below
    2^8), so every second-layer product is a multiple of 2^-16; with the absolute
    term sums below 2^14 and 2^8 (checked) every partial sum, in any order, is a
    binary32 number.  The two sides then hold the same activations and masks, and
    only the logit, dz and the backward sums round differently."""
    rng = np.random.default_rng(seed)
    p = M.init_params(rng, IN_DIM)
    p.W1[:IN_DIM] = rng.integers(-12, 13, (IN_DIM, M.HIDDEN)) * 2.0 ** -6
    p.b1[:] = rng.integers(-100, 101, M.HIDDEN) * 2.0 ** -10
    p.W2[:] = rng.integers(-4, 5, (M.HIDDEN, M.HIDDEN)) * 2.0 ** -6
    p.b2[:] = rng.integers(-3000, 3001, M.HIDDEN) * 2.0 ** -16
    p.b3[:] = 0.2
    x = (rng.integers(0, 16, (B, IN_DIM)) / 16.0).astype(np.float32)
    y = (rng.random(B) < 0.4).astype(np.float32)
    _, (X, Z1, A1, Z2, A2) = M.forward(p, x)
    on = lambda a, q: np.all(np.asarray(a, np.float64) * 2.0 ** q == np.round(np.asarray(a, np.float64) * 2.0 ** q))  # noqa: E731
    assert on(X, 4) and on(M.bf16(p.W1), 6) and on(p.b1, 10) and on(A1, 10)
    assert on(M.bf16(p.W2), 6) and on(p.b2, 16)
    assert np.max(np.abs(X) @ np.abs(M.bf16(p.W1)) + np.abs(p.b1)) < 2.0 ** 14
    assert np.max(np.abs(A1) @ np.abs(M.bf16(p.W2)) + np.abs(p.b2)) < 2.0 ** 8
    assert 0.2 < np.mean(Z1 > 0) < 0.8 and 0.2 < np.mean(Z2 > 0) < 0.8  # both masks live
    return p, x, y


@pytest.mark.parametrize("B", [200, 512])
def test_gradients_exact_forward(P, B):
    """On quantized_problem the forward pass is exact on both sides, so the
    element-wise bound is tight: about the binary32 rounding of the backward sums."""
    p, x, y = quantized_problem(50 + B, B)
    net = P.Mlp(IN_DIM, 512)
    net.set_params(flat(p))
    _, g = net.gradients(x, y)
    _, want, _ = M.loss_and_grads(p, x, y)
    gd = unflat(g)
    bounds = gradient_bounds(p, x, y, exact_forward=True)
    for k in M.PARAM_NAMES:
        ref = np.asarray(want[k], np.float64).reshape(gd[k].shape)
        bnd = 2.0 * bounds[k].reshape(gd[k].shape)
        err = np.abs(gd[k].astype(np.float64) - ref)
        over = np.nonzero(err > bnd)
        assert over[0].size == 0, (k, over[0][:5], err[over][:5], bnd[over][:5])


def test_gradient_bounds_catch_mistakes():
    """What the element-wise bounds see (a check of the test itself, on the host).
    On the exact-forward problem, a gradient that dropped one batch row of 200 fails
    the bound for most of the elements that row contributes to, in W2 and w3 (in
    W1, whose bound also carries the possible bfloat16 rounding changes of dZ1, for
    about a quarter of them).  The general bound is a
    worst case (a few per cent of the absolute term sums at the second layer, more
    at the first, where bfloat16 rounding changes of the activations compound), so
    there only gross element mistakes show: two 32-column blocks of W2's gradient
    swapped, or W2's or w3's gradient negated."""
    p, x, y = quantized_problem(31, 200)
    _, want, _ = M.loss_and_grads(p, x, y)
    _, short, _ = M.loss_and_grads(p, x[:-1], y[:-1])
    bounds = gradient_bounds(p, x, y, exact_forward=True)
    for k in ("W2", "w3"):
        ref = np.asarray(want[k], np.float64)
        wrong = np.asarray(short[k], np.float64) * (199.0 / 200.0)
        # where the dropped row's term is not 0 (ReLU masks); the rescaling's own
        # rounding is far below this cut
        moved = np.abs(wrong - ref) > 1e-9 * np.max(np.abs(ref))
        caught = np.abs(wrong - ref) > 2.0 * bounds[k]
        assert caught[moved].mean() > 0.5, (k, caught[moved].mean())
    p, x, y = problem(31, 200)
    _, want, _ = M.loss_and_grads(p, x, y)
    bounds = gradient_bounds(p, x, y)
    ref = np.asarray(want["W2"], np.float64)
    tile = ref.copy()
    tile[:, 0:32], tile[:, 32:64] = ref[:, 32:64].copy(), ref[:, 0:32].copy()
    nz = np.abs(ref) > 0
    nz[:, 64:] = False
    assert (np.abs(tile - ref) > 2.0 * bounds["W2"])[nz].mean() > 0.5
    for k in ("W2", "w3"):
        ref = np.asarray(want[k], np.float64)
        nz = np.abs(ref) > 0
        assert (np.abs(2.0 * ref) > 2.0 * bounds[k])[nz].mean() > 0.5, k


def test_zero_weights_closed_form(P):
    p, x, y = problem(7, 130)
    for k in ("W1", "b1", "W2", "b2", "w3"):
        getattr(p, k)[:] = 0.0
    p.b3[:] = 0.75
    net = P.Mlp(IN_DIM, 256)
    net.set_params(flat(p))
    assert np.all(net.forward(x) == np.float32(0.75))
    loss, g = net.gradients(x, y)
    gd = unflat(g)
    sig = 1.0 / (1.0 + np.exp(-0.75))
    assert abs(gd["b3"][0] - np.mean(sig - y)) < 1e-6
    for k in ("W1", "b1", "W2", "b2", "w3"):
        assert np.all(gd[k] == 0.0), k


def test_adam_against_oracle(P):
    """Three Adam steps on the device against oracle/mlp.py's Adam fed with the same
    gradients (the device's own, which test_gradients compares with the oracle's):
    the binary32 update is within a few ulps of the parameter plus a few ulps of the
    step size."""
    lr = 1e-3
    net = P.Mlp(IN_DIM, 256, lr=lr)
    p, _, _ = problem(8, 256)
    net.set_params(flat(p))
    opt = M.Adam(lr=lr)
    cur = p.copy()
    for step in range(3):
        _, x, y = problem(40 + step, 256)
        _, g = net.gradients(x, y)
        net.train_step(x, y)
        cur = opt.step(cur, unflat(g.astype(np.float64)))
        got = net.get_params().astype(np.float64)
        want = flat(cur).astype(np.float64)
        tol = 4.0 * U * np.abs(want) + 64.0 * U * lr * (step + 1) + 1e-30
        err = np.abs(got - want)
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, (step, bad[:5], got[bad[:5]], want[bad[:5]])


def test_adam_step_and_training(P):
    """A learnable rule: the label is whether x0 + x1 > 1."""
    rng = np.random.default_rng(9)
    xs = rng.random((4096, IN_DIM)).astype(np.float32)
    ys = (xs[:, 0] + xs[:, 1] > 1.0).astype(np.float32)
    net2 = P.Mlp(IN_DIM, 512, lr=2e-3)
    net2.set_params(flat(M.init_params(np.random.default_rng(1), IN_DIM)))
    losses = []
    for step in range(300):
        i = (step * 512) % 4096
        losses.append(net2.train_step(xs[i:i + 512], ys[i:i + 512]))
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20]), (losses[:3], losses[-3:])
    acc = np.mean((net2.forward(xs[:512]) > 0) == (ys[:512] > 0))
    assert acc > 0.9, acc


def test_mlp_invalid_arguments(P):
    with pytest.raises(P.PirrtError):
        P.Mlp(0, 10)
    with pytest.raises(P.PirrtError):
        P.Mlp(300, 10)
    net = P.Mlp(IN_DIM, 64)
    with pytest.raises(P.PirrtError):
        net.forward(np.zeros((65, IN_DIM), np.float32))
    bad = np.zeros(net.num_params, np.float32)
    bad[5] = np.nan
    with pytest.raises(P.PirrtError):
        net.set_params(bad)
