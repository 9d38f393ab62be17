"""Pins of the learned-proposal network's oracle (oracle/mlp.py): bfloat16 rounding
against torch's conversion and hand-worked ties, the backward pass against torch
autograd and FP64 central differences, closed forms at zero weights, the first
Adam step, and the label rule."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, -2.5, 3.0e38, 1e-40, 0.0, np.inf])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -2.5, np.float32(3.0e38), 1e-40, 0.0, np.inf])
    got = M.bf16(x)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(got[:6], M.bf16(want[:6]))
    assert got[1] == 1.0 and got[2] == 1 + 2.0 ** -6  # ties to even
    rng = np.random.default_rng(0)
    r = rng.standard_normal(10000) * 10.0 ** rng.integers(-20, 20, 10000)
    assert np.array_equal(M.bf16(r), torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).double().numpy())


def small_problem(seed=1, B=6):
    rng = np.random.default_rng(seed)
    p = M.init_params(rng, 286)
    p.b1[:] = rng.standard_normal(M.HIDDEN) * 0.1
    p.b2[:] = rng.standard_normal(M.HIDDEN) * 0.1
    p.b3[:] = 0.3
    f = rng.random((B, 286))
    y = (rng.random(B) < 0.5).astype(np.float32)
    return p, f, y


def test_backward_matches_torch_autograd():
    p, f, y = small_problem()
    loss, g, z = M.loss_and_grads(p, f, y, exact=True)
    t = {k: torch.tensor(v.astype(np.float64), requires_grad=True) for k, v in p.as_dict().items()}
    X = torch.tensor(M.pad_features(f))
    h1 = torch.relu(X @ t["W1"] + t["b1"])
    h2 = torch.relu(h1 @ t["W2"] + t["b2"])
    zt = h2 @ t["w3"] + t["b3"][0]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.tensor(y, dtype=torch.float64))
    lt.backward()
    assert abs(lt.item() - loss) < 1e-12 * max(1.0, abs(loss))
    assert np.allclose(zt.detach().numpy(), z, rtol=1e-12, atol=1e-12)
    for k in M.PARAM_NAMES:
        ref = t[k].grad.numpy()
        assert np.allclose(g[k], ref, rtol=1e-10, atol=1e-14), k


def test_backward_central_differences():
    p, f, y = small_problem(seed=2, B=4)
    _, g, _ = M.loss_and_grads(p, f, y, exact=True)
    rng = np.random.default_rng(3)
    h = 1e-6
    for k in M.PARAM_NAMES:
        arr = getattr(p, k)
        idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
        for i in idx:
            if k == "W1" and i[0] >= 286:
                continue
            q = p.copy()
            qa = {kk: vv.astype(np.float64) for kk, vv in q.as_dict().items()}
            base = qa[k][i]
            qa[k][i] = base + h
            lp = M.loss_and_grads(M.Params(**qa), f, y, exact=True)[0]
            qa[k][i] = base - h
            lm = M.loss_and_grads(M.Params(**qa), f, y, exact=True)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, g[k][i])


def test_zero_weights_closed_form():
    p, f, y = small_problem(seed=4, B=8)
    for k in ("W1", "b1", "W2", "b2", "w3"):
        getattr(p, k)[:] = 0.0
    p.b3[:] = 0.75
    loss, g, z = M.loss_and_grads(p, f, y)
    assert np.all(z == 0.75)
    sig = 1.0 / (1.0 + np.exp(-0.75))
    assert abs(loss - np.mean(np.where(y > 0, np.log1p(np.exp(-0.75)), 0.75 + np.log1p(np.exp(-0.75))))) < 1e-12
    assert abs(g["b3"][0] - np.mean(sig - y)) < 1e-12
    for k in ("W1", "b1", "W2", "b2", "w3"):
        assert np.all(g[k] == 0.0), k
    assert abs(M.bce_with_logits(np.zeros(3), np.array([0.0, 1.0, 1.0])) - np.log(2.0)) < 1e-15


def test_adam_first_step_is_signed_lr():
    p, f, y = small_problem(seed=5)
    _, g, _ = M.loss_and_grads(p, f, y)
    opt = M.Adam(lr=1e-3)
    q = opt.step(p, g)
    for k in M.PARAM_NAMES:
        gk = np.asarray(g[k], np.float64)
        want = p.as_dict()[k].astype(np.float64) - 1e-3 * gk / (np.abs(gk) + 1e-8)
        assert np.allclose(getattr(q, k), want.astype(np.float32), rtol=0, atol=1e-7), k


def test_labels_rule():
    g_r = np.array([0.0, 10.0, 3.0, 6.0, np.inf, 9.0], np.float32)
    g_t = np.array([10.0, 0.0, 7.0, 4.6, 1.0, 1.4], np.float32)
    # totals: 10, 10, 10, 10.6, inf, 10.4 against 1.05 * 10 = 10.5
    assert np.array_equal(M.labels(g_r, g_t), np.array([1, 1, 1, 0, 0, 1], np.float32))


def test_features_layout():
    class Obs:
        d = 2
        kind = np.array([0, 1, 0], np.int32)
        centre = np.array([[0.1, 0.2], [0.5, 0.5], [0.7, 0.8]])
        size = np.array([[0.05, 0.0], [0.1, 0.1], [0.06, 0.0]])
    enc = M.obstacle_encoding(Obs(), n_slots=3)
    assert np.array_equal(enc, [0.1, 0.2, 0.05, 0.7, 0.8, 0.06, 0.0, 0.0, 0.0])
    f = M.features(np.array([[0.3, 0.4]]), enc)
    assert f.shape == (1, 11) and np.array_equal(f[0, :2], [0.3, 0.4])
