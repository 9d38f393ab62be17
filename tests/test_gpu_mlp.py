"""The learned proposal's network on the device (pirrt_mlp_* through the C ABI)
against the oracle (oracle/mlp.py).

Tolerance, from the arithmetic: both sides use the same bfloat16 inputs and weights
and exact products; only the accumulation differs (binary32 on the device, binary64
in the oracle).  An activation can therefore differ by one bfloat16 ulp (2^-8
relative) where the two sums fall on opposite sides of a rounding boundary, and such a
difference moves the logit by at most 2^-8 times the absolute path sum downstream of
it.  The bound used is twice that sum over every activation (accumulation error
included), per logit; the median error must also be far below it, so a systematic
mistake (a wrong lane layout, a dropped bias) cannot hide under the bound."""
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


@pytest.mark.parametrize("B", [64, 200, 512])
def test_gradients(P, B):
    p, x, y = problem(20 + B, B)
    net = P.Mlp(IN_DIM, 512)
    net.set_params(flat(p))
    loss, g = net.gradients(x, y)
    want_loss, want, _ = M.loss_and_grads(p, x, y)
    assert abs(loss - want_loss) <= 1e-3 * abs(want_loss) + 1e-5
    gd = unflat(g)
    for k in M.PARAM_NAMES:
        ref = np.asarray(want[k], np.float64)
        diff = np.linalg.norm(gd[k] - ref)
        assert diff <= 2.0 ** -6 * np.linalg.norm(ref) + 1e-7, (k, diff, np.linalg.norm(ref))
    assert np.all(gd["W1"][IN_DIM:] == 0.0)  # padding rows of X are zero


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


def test_adam_step_and_training(P):
    p, x, y = problem(8, 256)
    lr = 1e-3
    net = P.Mlp(IN_DIM, 256, lr=lr)
    net.set_params(flat(p))
    _, g = net.gradients(x, y)
    before = net.get_params()
    net.train_step(x, y)
    after = net.get_params()
    # first Adam step: p - lr * g / (|g| + eps) with the device's own gradient
    want = before.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(after - want)) <= 1e-6
    # a learnable rule: the label is whether x0 + x1 > 1
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
