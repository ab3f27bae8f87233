"""Parity of the warm-start network's GPU kernels (matrix-core inference, training gradient,
AdamW) with the FP64 oracle, through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import mlp as M
from paper_2606_28394_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def J():
    from paper_2606_28394_amd import jenga
    jenga.load_library()
    return jenga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(seed):
    """Random parameters with bfloat16-representable weights and a non-trivial normalisation."""
    flat = W.mlp_init(seed)
    P = M.unpack(flat)
    rng = np.random.default_rng(100 + seed)
    P["mean"][:] = rng.normal(0.0, 0.5, 24)
    P["std"][:] = rng.uniform(0.5, 2.0, 24)
    flat[:M.N_TRAINABLE] = M.bf16(flat[:M.N_TRAINABLE])
    return flat.astype(np.float32).astype(np.float64)


def _features(n, seed):
    P = np.random.default_rng(200 + seed)
    F = W.random_features(n, seed) * P.uniform(0.5, 2.0, 24) + P.normal(0.0, 0.5, 24)
    return F.astype(np.float32).astype(np.float64)


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_forward_matches_oracle(J, n):
    import torch
    flat = _params(1)
    F = _features(n, 1)
    net = J.Mlp(flat)
    y = net.forward(_dev(torch, F)).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(flat, F, rounding=True)
    scale = np.sqrt(np.mean(ref ** 2))
    err = np.abs(y - ref)
    _say(f"forward n={n}: max|dy| {err.max():.3e}, rms(y) {scale:.3e}")
    # bf16 layer inputs: an FP32 vs FP64 difference can flip a rounding (one bf16 ulp, 2^-8)
    assert np.all(err <= 1e-2 * np.maximum(np.abs(ref), scale))
    assert err.max() <= 2e-3 * max(np.abs(ref).max(), 1.0)


def test_forward_large_batch_sampled(J):
    import torch
    flat = _params(2)
    n = 200_003
    F = _features(n, 2)
    net = J.Mlp(flat)
    y = net.forward(_dev(torch, F)).cpu().numpy().astype(np.float64)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(n - 67, n),
                                    np.random.default_rng(3).choice(n, 2000, replace=False)]))
    ref, _ = M.forward(flat, F[idx], rounding=True)
    scale = np.sqrt(np.mean(ref ** 2))
    assert np.all(np.abs(y[idx] - ref) <= 1e-2 * np.maximum(np.abs(ref), scale))


@pytest.mark.parametrize("n", [1, 65, 1000, 40_000])
def test_gradient_matches_oracle(J, n):
    import torch
    flat = _params(3)
    F = _features(n, 3)
    T = np.random.default_rng(4).standard_normal((n, 3)).astype(np.float32).astype(np.float64)
    net = J.Mlp(flat)
    g, loss = net.compute_grad(_dev(torch, F), _dev(torch, T))
    g = g.cpu().numpy().astype(np.float64)
    y, cache = M.forward(flat, F, rounding=True)
    ref = M.backward(flat, cache, y, T)[:M.N_TRAINABLE]
    assert float(loss.item()) == pytest.approx(M.mse(y, T), rel=2e-3)
    o = 0
    for name, shape in M.LAYOUT[:6]:
        k = int(np.prod(shape))
        a, b = g[o:o + k], ref[o:o + k]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        _say(f"grad n={n} {name}: rel {rel:.3e}, max|g| {np.abs(b).max():.3e}")
        assert rel < 1e-2, name
        assert np.abs(a - b).max() <= 1e-2 * np.abs(b).max() + 1e-12, name
        o += k


def test_gradient_is_deterministic(J):
    import torch
    flat = _params(4)
    F = _dev(torch, _features(5000, 4))
    T = _dev(torch, np.random.default_rng(5).standard_normal((5000, 3)))
    net = J.Mlp(flat)
    g1 = net.compute_grad(F, T)[0].clone()
    g2 = net.compute_grad(F, T)[0].clone()
    assert torch.equal(g1, g2)


def test_adamw_matches_oracle(J):
    import torch
    flat = _params(5)
    net = J.Mlp(flat)
    opt = M.AdamW(lr=1e-3, weight_decay=1e-2)
    ref = flat.copy()
    rng = np.random.default_rng(6)
    for _ in range(4):
        g = rng.standard_normal(M.SIZE) * 1e-2
        g[M.N_TRAINABLE:] = 0.0
        g32 = g.astype(np.float32).astype(np.float64)
        net.grad.copy_(torch.as_tensor(g32[:M.N_TRAINABLE], dtype=torch.float32))
        net.adamw(lr=1e-3, weight_decay=1e-2)
        opt.step(ref, g32)
    got = net.params.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got[:M.N_TRAINABLE], ref[:M.N_TRAINABLE], rtol=1e-5, atol=1e-7)
    np.testing.assert_array_equal(got[M.N_TRAINABLE:], flat[M.N_TRAINABLE:].astype(np.float32))


def test_training_reduces_loss(J):
    import torch
    n = 4096
    F = _features(n, 7)
    T = np.stack([np.tanh(F[:, 0]), 0.5 * F[:, 1] * F[:, 2], 0.3 * F[:, 3]], axis=1)
    flat = W.mlp_init(7)
    P = M.unpack(flat)
    P["mean"][:], P["std"][:] = M.normalisation(F)
    net = J.Mlp(flat)
    Fd, Td = _dev(torch, F), _dev(torch, T)
    first = None
    for _ in range(300):
        loss = float(net.train_step(Fd, Td, lr=3e-3).item())
        first = loss if first is None else first
    _say(f"training: loss {first:.4f} -> {loss:.4f}")
    assert loss < 0.2 * first
