"""pirrt_mlp_forward_noalloc (the forward pass that allocates nothing: its scratch is
a fixed device array of the library) against pirrt_mlp_forward, through the C ABI.

Both run the same kernels on the same bfloat16 operands, so the logits must agree bit
for bit.  Two calls in a row, the second with a smaller batch, check that the array
keeps nothing from one call that the next one reads: a stale row of the first call
would show in the second's logits.  The logits of both are also held to the oracle's
(oracle/mlp.py) within the bound derived in test_gpu_mlp.py."""
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


def logit_bound(p, x):
    _, (X, Z1, A1, Z2, A2) = M.forward(p, x)
    aw3 = np.abs(M.bf16(p.w3))
    down1 = np.abs(M.bf16(p.W2)) @ aw3
    return 2.0 * 2.0 ** -8 * (np.abs(A2) @ aw3 + np.abs(A1) @ down1) + 1e-6


def test_noalloc_forward_matches_forward(P):
    import torch
    rng = np.random.default_rng(4242)
    p = M.init_params(rng, IN_DIM)
    p.b1[:] = (rng.standard_normal(M.HIDDEN) * 0.1).astype(np.float32)
    p.b2[:] = (rng.standard_normal(M.HIDDEN) * 0.1).astype(np.float32)
    p.b3[:] = -0.3
    stream = torch.cuda.current_stream()
    net = P.Mlp(IN_DIM, P.PIRRT_MLP_NOALLOC_MAX_BATCH, stream=stream.cuda_stream)
    net.set_params(flat(p))
    # the largest batch first (every row of the array in use), then a smaller, ragged one
    for B, seed in ((P.PIRRT_MLP_NOALLOC_MAX_BATCH, 1), (777, 2)):
        x = np.random.default_rng(seed).random((B, IN_DIM)).astype(np.float32)
        xd = torch.from_numpy(x).cuda()
        want = net.forward(xd).cpu().numpy()
        got = torch.full((B + 64,), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(xd, got[:B])
        stream.synchronize()
        got = got.cpu().numpy()
        assert np.array_equal(got[:B].view(np.uint32), want.view(np.uint32)), B
        assert np.all(np.isnan(got[B:])), "wrote past the B logits"
        ref, _ = M.forward(p, x)
        assert np.all(np.abs(got[:B] - ref) <= logit_bound(p, x)), B


def test_noalloc_forward_rejects_sizes(P):
    import torch
    net = P.Mlp(IN_DIM, 64)
    x = torch.zeros((P.PIRRT_MLP_NOALLOC_MAX_BATCH + 1, IN_DIM), dtype=torch.float32, device="cuda")
    out = torch.zeros(P.PIRRT_MLP_NOALLOC_MAX_BATCH + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PirrtError) as e:
        net.forward_noalloc(x, out)
    assert e.value.code == P.PIRRT_EINVAL
    with pytest.raises(P.PirrtError) as e:
        net.forward_noalloc(x[:0], out[:0])
    assert e.value.code == P.PIRRT_EINVAL
    # the handle stays usable after the rejected calls
    net.forward_noalloc(x[:5], out[:5])
    torch.cuda.synchronize()
    assert torch.all(out[:5] == 0.0)
