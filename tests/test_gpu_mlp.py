"""The controller network's matrix-core kernels against the FP64 network
oracle: the BF16 GEMM on ragged and strided shapes, the forward pass, every
parameter gradient, one Adam step, and a short fit that must lower the loss.

Tolerances: both sides round the same FP32 operands to BF16, so what is left
is FP32 accumulation (K <= 1024 terms: below 1e-5 of sum |a b|) and, past the
first layer, activations that sit within an FP32 rounding of a BF16 rounding
boundary (rare, each moving one operand by 2^-8 relative)."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo
from paper_1806_10589_amd import fluxlbm, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device=DEV)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (16, 16, 16), (37, 21, 50), (130, 128, 32), (5, 128, 1000)])
def test_gemm_bf16_matches_rounded_fp64(m, n, k):
    a = inputs.uniform_noise((m, k), 100 + m)
    b = inputs.uniform_noise((k, n), 200 + n)
    c = torch.full((m, n), float("nan"), device=DEV)
    A, B = _t(a), _t(b)
    fluxlbm.flbm_gemm_bf16(A.data_ptr(), k, 1, B.data_ptr(), n, 1, c.data_ptr(), n, m, n, k,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = mo.round_bf16(a) @ mo.round_bf16(b)
    # FP32 accumulation of k terms: at most k 2^-24 of sum |a b|
    bound = (k * 2.0 ** -24 + 1e-7) * (np.abs(mo.round_bf16(a)) @ np.abs(mo.round_bf16(b))) + 1e-30
    got = c.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= bound)


def test_gemm_bf16_strided_operands():
    # A given transposed (column-major), B a row slice with a wide stride
    m, n, k = 23, 19, 45
    a = inputs.uniform_noise((k, m), 7)          # stored as A^T
    b = inputs.uniform_noise((k, 3 * n), 8)      # use every third column
    c = torch.zeros((m, n + 5), device=DEV)
    A, B = _t(a), _t(b)
    fluxlbm.flbm_gemm_bf16(A.data_ptr(), 1, m, B.data_ptr(), 3 * n, 3, c.data_ptr(), n + 5, m, n, k,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = mo.round_bf16(a.T) @ mo.round_bf16(b[:, ::3])
    got = c.cpu().numpy()
    assert np.allclose(got[:, :n], ref, rtol=0, atol=1e-5 * np.abs(ref).max())
    assert not np.any(got[:, n:])  # the padding columns are untouched


def _net(seed, scale=0.3, batch=512):
    net = fluxlbm.Mlp(batch)
    p = (scale * inputs.uniform_noise((mo.N_PARAMS,), seed)).astype(np.float32)
    net.set_params(p)
    return net, p.astype(np.float64)


@pytest.mark.parametrize("batch", [1, 17, 300])
def test_forward_matches_oracle(batch):
    net, p = _net(41)
    x = inputs.uniform_noise((batch, 32), 42)
    y = net.forward(_t(x)).cpu().numpy()
    yo, _, _ = mo.forward(p, x.astype(np.float32), bf16=True)
    assert np.max(np.abs(y - yo)) <= 2e-4 * max(1.0, np.abs(yo).max())
    net.close()


def test_gradients_match_oracle():
    net, p = _net(51)
    x = inputs.uniform_noise((200, 32), 52).astype(np.float32)
    t = inputs.uniform_noise((200,), 53).astype(np.float32)
    g, loss = net.gradients(_t(x), _t(t))
    lo, go = mo.gradients(p, x, t, bf16=True)
    assert loss == pytest.approx(lo, rel=1e-4)
    # every block to 1e-3 of its own largest entry
    o = 0
    for name, shape in mo.SHAPES:
        k = int(np.prod(shape))
        gb, ob = g[o:o + k], go[o:o + k]
        assert np.max(np.abs(gb - ob)) <= 1e-3 * np.abs(ob).max() + 1e-7, name
        o += k
    # and the unrounded FP64 gradient is within BF16 accuracy
    _, ge = mo.gradients(p, x, t)
    assert np.max(np.abs(g - ge)) <= 0.03 * np.abs(ge).max()
    net.close()


def test_adam_step_matches_oracle():
    net, p = _net(61)
    x = inputs.uniform_noise((64, 32), 62).astype(np.float32)
    t = inputs.uniform_noise((64,), 63).astype(np.float32)
    g, _ = net.gradients(_t(x), _t(t))
    lr = 1e-3
    net.train_step(_t(x), _t(t), lr)
    p1 = net.get_params().astype(np.float64)
    # the same update from the device's own gradient, in FP64
    pe, _, _ = mo.adam_step(p, g.astype(np.float64), np.zeros_like(p), np.zeros_like(p), 1, lr)
    assert np.max(np.abs(p1 - pe)) <= 1e-6
    # and, from the oracle's gradient, the step is lr sign(g) except where g is tiny
    _, go = mo.gradients(p, x, t, bf16=True)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.allclose((p1 - p)[big], -lr * np.sign(go[big]), rtol=1e-3, atol=1e-7)
    net.close()


def test_training_lowers_the_loss():
    # a smooth target of a few inputs
    x = inputs.uniform_noise((2048, 32), 71).astype(np.float32)
    t = (np.sin(2 * x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]).astype(np.float32)
    net = fluxlbm.Mlp(256)
    net.set_params((0.1 * inputs.uniform_noise((mo.N_PARAMS,), 72)).astype(np.float32))
    X, T = _t(x), _t(t)
    g = torch.Generator(device=DEV)
    g.manual_seed(0)
    first = None
    for i in range(600):
        idx = torch.randint(0, 2048, (256,), device=DEV, generator=g)
        loss = net.train_step(X[idx], T[idx], 3e-3, want_loss=(i == 0))
        if i == 0:
            first = loss
    _, final = net.gradients(X[:256], T[:256])
    assert final < 0.1 * first
    net.close()


def test_invalid_batch_rejected():
    net = fluxlbm.Mlp(8)
    with pytest.raises(fluxlbm.FlbmError):
        net.forward(_t(np.zeros((9, 32))))
    with pytest.raises(fluxlbm.FlbmError):
        fluxlbm.flbm_mlp_set_params(net.handle, np.zeros(10, np.float32))
    net.close()
