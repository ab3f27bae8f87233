"""Pins of the warm-start network oracle (numpy and C) against closed forms, finite
differences and independent library routines (torch on the CPU, in float64)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import oracle as O
from paper_2606_28394_amd import workloads as W


def _torch_net(flat):
    P = M.unpack(flat)
    net = torch.nn.Sequential(torch.nn.Linear(24, 128), torch.nn.GELU(approximate="none"),
                              torch.nn.Linear(128, 128), torch.nn.GELU(approximate="none"),
                              torch.nn.Linear(128, 3)).double()
    with torch.no_grad():
        for lin, w, b in ((net[0], "W1", "b1"), (net[2], "W2", "b2"), (net[4], "W3", "b3")):
            lin.weight.copy_(torch.from_numpy(P[w].T.copy()))   # torch stores [out][in]
            lin.bias.copy_(torch.from_numpy(P[b].copy()))
    return net


def _scaled_params(seed=0):
    flat = W.mlp_init(seed)
    P = M.unpack(flat)
    rng = np.random.default_rng(seed + 7)
    P["mean"][:] = rng.normal(0.0, 0.5, 24)
    P["std"][:] = rng.uniform(0.5, 2.0, 24)
    return flat


def test_layout_size():
    assert M.N_TRAINABLE == 20099
    assert M.SIZE == O.MLP_SIZE


def test_bf16_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-30, 30, 4000),
                        [0.0, -0.0, 1.0, -1.0, 1.00390625, 1.0078125, 1.01171875, 3.4e38, -3.4e38, 1e-40]])
    ref = torch.from_numpy(x).float().to(torch.bfloat16).double().numpy()
    got = M.bf16(x)
    np.testing.assert_array_equal(got, ref)
    got_c = np.array([O.bf16(v) for v in x[:600]] + [O.bf16(v) for v in x[-10:]])
    np.testing.assert_array_equal(got_c, np.concatenate([ref[:600], ref[-10:]]))


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: rounds to the even mantissa (1.0);
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: rounds up to the even one
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_gelu_closed_forms():
    # x Phi(x) at 1 and 2 (Phi from the complementary error function's tabulated values)
    assert M.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array(2.0)) == pytest.approx(2.0 * 0.9772498680518208, rel=1e-15)
    assert M.gelu(np.array(0.0)) == 0.0
    x = np.linspace(-6, 6, 121)
    np.testing.assert_allclose(M.gelu(-x), M.gelu(x) - x, atol=1e-15)     # Phi(-x) = 1 - Phi(x)
    np.testing.assert_allclose(M.gelu(x), torch.nn.functional.gelu(torch.from_numpy(x)).numpy(), rtol=1e-15,
                               atol=1e-16)


def test_gelu_grad_central_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-5
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), fd, rtol=1e-9, atol=1e-11)
    assert M.gelu_grad(np.array(0.0)) == 0.5


def test_forward_matches_torch_modules():
    flat = _scaled_params(1)
    F = W.random_features(64, 1)
    y, _ = M.forward(flat, F, rounding=False)
    P = M.unpack(flat)
    with torch.no_grad():
        ref = _torch_net(flat)(torch.from_numpy((F - P["mean"]) / P["std"])).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-14)


def test_forward_rounded_matches_torch_bf16_steps():
    """Rounded forward against torch ops with explicit bfloat16 casts between layers."""
    flat = M.bf16(_scaled_params(2))
    P = M.unpack(flat)
    F = W.random_features(64, 2)
    y, _ = M.forward(flat, F, rounding=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    rb = lambda a: a.float().to(torch.bfloat16).double()
    x0 = rb((t(F) - t(P["mean"])) / t(P["std"]))
    h1 = rb(torch.nn.functional.gelu(x0 @ t(P["W1"]) + t(P["b1"])))
    h2 = rb(torch.nn.functional.gelu(h1 @ t(P["W2"]) + t(P["b2"])))
    ref = (h2 @ t(P["W3"]) + t(P["b3"])).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-14)


def test_c_forward_matches_numpy():
    flat = M.bf16(_scaled_params(3))
    F = W.random_features(50, 3)
    y, _ = M.forward(flat, F, rounding=True)
    yc = np.array([O.mlp_forward(flat, f) for f in F])
    np.testing.assert_allclose(yc, y, rtol=1e-12, atol=1e-13)


def test_backward_finite_differences():
    """Analytic gradient against central differences, relative error < 1e-7 per checked entry."""
    flat = _scaled_params(4)
    F = W.random_features(16, 4)
    tgt = np.random.default_rng(4).standard_normal((16, 3))
    y, cache = M.forward(flat, F, rounding=False)
    g = M.backward(flat, cache, y, tgt)
    rng = np.random.default_rng(5)
    offsets, o = {}, 0
    for name, shape in M.LAYOUT:
        offsets[name] = (o, int(np.prod(shape)))
        o += int(np.prod(shape))
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        start, n = offsets[name]
        for idx in rng.choice(n, size=min(n, 12), replace=False):
            i = start + int(idx)
            h = 1e-3 * max(1.0, abs(flat[i]))

            def loss_at(delta):
                f = flat.copy()
                f[i] += delta
                return M.mse(M.forward(f, F, False)[0], tgt)
            # fourth-order central stencil (truncation ~h^4, cancellation ~1e-16 / h)
            fd = (-loss_at(2 * h) + 8 * loss_at(h) - 8 * loss_at(-h) + loss_at(-2 * h)) / (12 * h)
            assert abs(g[i] - fd) <= 1e-7 * max(abs(fd), 1e-6), (name, idx, g[i], fd)
    np.testing.assert_array_equal(g[M.N_TRAINABLE:], 0.0)


def test_backward_matches_autograd():
    flat = _scaled_params(5)
    P = M.unpack(flat)
    F = W.random_features(32, 5)
    tgt = np.random.default_rng(6).standard_normal((32, 3))
    y, cache = M.forward(flat, F, rounding=False)
    g = M.unpack(M.backward(flat, cache, y, tgt))
    net = _torch_net(flat)
    loss = torch.nn.functional.mse_loss(net(torch.from_numpy((F - P["mean"]) / P["std"])), torch.from_numpy(tgt))
    loss.backward()
    assert loss.item() == pytest.approx(M.mse(y, tgt), rel=1e-13)
    for lin, w, b in ((net[0], "W1", "b1"), (net[2], "W2", "b2"), (net[4], "W3", "b3")):
        np.testing.assert_allclose(g[w], lin.weight.grad.numpy().T, rtol=1e-11, atol=1e-15)
        np.testing.assert_allclose(g[b], lin.bias.grad.numpy(), rtol=1e-11, atol=1e-15)


def test_adamw_matches_torch():
    flat = _scaled_params(6)
    P = M.unpack(flat)
    F = W.random_features(32, 6)
    tgt = np.random.default_rng(7).standard_normal((32, 3))
    net = _torch_net(flat)
    params = [net[0].weight, net[0].bias, net[2].weight, net[2].bias, net[4].weight, net[4].bias]
    opt_t = torch.optim.AdamW(params, lr=3e-3, weight_decay=1e-2)
    opt = M.AdamW(lr=3e-3, weight_decay=1e-2)
    xin = torch.from_numpy((F - P["mean"]) / P["std"])
    for _ in range(5):
        y, cache = M.forward(flat, F, rounding=False)
        opt.step(flat, M.backward(flat, cache, y, tgt))
        opt_t.zero_grad()
        torch.nn.functional.mse_loss(net(xin), torch.from_numpy(tgt)).backward()
        opt_t.step()
    Q = M.unpack(flat)
    for lin, w, b in ((net[0], "W1", "b1"), (net[2], "W2", "b2"), (net[4], "W3", "b3")):
        np.testing.assert_allclose(Q[w], lin.weight.detach().numpy().T, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(Q[b], lin.bias.detach().numpy(), rtol=1e-10, atol=1e-13)


def test_training_reduces_loss():
    flat = W.mlp_init(7)
    F = W.random_features(256, 7)
    tgt = np.stack([np.sin(F[:, 0]), F[:, 1] * F[:, 2], 0.5 * F[:, 3]], axis=1)
    opt = M.AdamW(lr=3e-3)
    first = None
    for _ in range(150):
        y, cache = M.forward(flat, F, rounding=False)
        first = first if first is not None else M.mse(y, tgt)
        opt.step(flat, M.backward(flat, cache, y, tgt))
    assert M.mse(M.forward(flat, F, rounding=False)[0], tgt) < 0.25 * first


def test_warm_start_mapping():
    k = np.array([[200.0, 400.0, 500.0], [100.0, 100.0, 100.0], [100.0, 100.0, 100.0]])
    y = np.array([[2.0, 10.0, -0.5], [-1.0, 3.0, 3.0], [-1.0, 0.5, 0.0]])
    prev = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [3.0, -0.5, 0.25]])
    g, dt, mu = 9.81, 1 / 240, 0.4
    lam = M.warm_start(y, k, prev, mu, g, dt)
    gdt = g * dt
    np.testing.assert_allclose(lam[0], [2 * gdt / 200, mu * 2 * gdt / 200, -0.5 * gdt / 500])
    np.testing.assert_array_equal(lam[1], [0.0, 0.0, 0.0])   # a pulling normal clamps all three
    np.testing.assert_allclose(lam[2], [2 * gdt / 100, 0.0, 0.25 * gdt / 100])   # outputs add to prev
    np.testing.assert_allclose(M.targets(k, lam, prev, g, dt)[2], [-1.0, 0.5, 0.0], atol=1e-12)
