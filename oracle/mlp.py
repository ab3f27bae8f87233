"""FP64 oracle of the learned warm start's per-contact network.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the benchmark's
CPU-baseline leg.  The product path never imports this module.

Network (learned warm start of the contact solver): 24 contact features, z-scored
with training-set statistics, then Linear(24, 128) -> GELU -> Linear(128, 128) -> GELU
-> Linear(128, 3).  GELU is the exact form x * Phi(x).  The three outputs are the change
of the dimensionless impulses lambda_d * k_d / (|g| dt) (d = normal, t1, t2; k_d the row's
inverse effective mass, Eq. (keff)) from the previous step's, which are input features
12..14; training minimises their mean squared error against a converged plain solve, with
AdamW (the paper's optimiser defaults: learning rate 3e-4, weight decay 1e-4).

Parameters live in one flat float64 vector, in this order (the same as the C oracle's
``or_mlp_forward``): W1[24][128], b1[128], W2[128][128], b2[128], W3[128][3], b3[3],
mean[24], std[24].  W[i][j] multiplies input i into output j.  The first 20,099
entries are trainable; mean and std are the fixed normalisation.

``rounding=True`` rounds each layer's input to bfloat16 (round to nearest even), as the
GPU feeds its matrix cores; the caller rounds the weights.  Gradients treat that
rounding as the identity; the finite-difference checks run with ``rounding=False``.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NFEAT, HIDDEN, NOUT = 24, 128, 3
LAYOUT = (("W1", (NFEAT, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, NOUT)), ("b3", (NOUT,)), ("mean", (NFEAT,)), ("std", (NFEAT,)))
SIZE = sum(int(np.prod(s)) for _, s in LAYOUT)
N_TRAINABLE = SIZE - 2 * NFEAT
SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def unpack(flat: np.ndarray) -> dict:
    """Views of the named blocks of a flat parameter vector."""
    assert flat.size == SIZE
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(blocks: dict) -> np.ndarray:
    return np.concatenate([np.asarray(blocks[name], np.float64).reshape(-1) for name, _ in LAYOUT])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (via single precision, then nearest even on the float's bits)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).copy()
    finite = (u & np.uint32(0x7F800000)) != np.uint32(0x7F800000)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    u = np.where(finite, r, u)
    return u.view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(flat: np.ndarray, feats: np.ndarray, rounding: bool = True):
    """Outputs (B, 3) for features (B, 24), and the cache the backward pass needs."""
    P = unpack(np.asarray(flat, np.float64))
    x0 = (np.asarray(feats, np.float64) - P["mean"]) / P["std"]
    rnd = bf16 if rounding else (lambda a: a)
    x0 = rnd(x0)
    z1 = x0 @ P["W1"] + P["b1"]
    h1 = rnd(gelu(z1))
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = rnd(gelu(z2))
    y = h2 @ P["W3"] + P["b3"]
    return y, dict(x0=x0, z1=z1, h1=h1, z2=z2, h2=h2)


def mse(y: np.ndarray, target: np.ndarray) -> float:
    """Mean over the batch and the three outputs of the squared error."""
    return float(np.mean((y - target) ** 2))


def backward(flat: np.ndarray, cache: dict, y: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Gradient of ``mse(y, target)`` with respect to the flat vector (zeros for mean and std)."""
    P = unpack(np.asarray(flat, np.float64))
    B = y.shape[0]
    dy = 2.0 * (y - target) / (B * NOUT)
    g = {name: np.zeros(shape) for name, shape in LAYOUT}
    g["W3"] = cache["h2"].T @ dy
    g["b3"] = dy.sum(axis=0)
    dz2 = (dy @ P["W3"].T) * gelu_grad(cache["z2"])
    g["W2"] = cache["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"].T) * gelu_grad(cache["z1"])
    g["W1"] = cache["x0"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


class AdamW:
    """Decoupled weight decay Adam (Loshchilov and Hutter), bias-corrected moments:
    p <- p (1 - lr wd); m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    Applied to the trainable entries only."""

    def __init__(self, lr=3e-4, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-4):
        self.lr, self.b1, self.b2, self.eps, self.wd = lr, betas[0], betas[1], eps, weight_decay
        self.m = np.zeros(N_TRAINABLE)
        self.v = np.zeros(N_TRAINABLE)
        self.t = 0

    def step(self, flat: np.ndarray, grad: np.ndarray) -> None:
        self.t += 1
        p = flat[:N_TRAINABLE]
        g = grad[:N_TRAINABLE]
        p *= 1.0 - self.lr * self.wd
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        p -= self.lr * mhat / (np.sqrt(vhat) + self.eps)


def normalisation(feats: np.ndarray, floor: float = 1e-12):
    """Training-set mean and standard deviation per feature (a constant feature gets std 1)."""
    mean = feats.mean(axis=0)
    std = feats.std(axis=0)
    return mean, np.where(std > floor, std, 1.0)


def targets(k: np.ndarray, lam: np.ndarray, prev: np.ndarray, gravity_norm: float, dt: float) -> np.ndarray:
    """Training targets: the change lambda_d k_d / (|g| dt) - prev_d of the dimensionless impulses
    from the previous step's (prev = features 12..14)."""
    return lam * k / (gravity_norm * dt) - prev


def warm_start(y: np.ndarray, k: np.ndarray, prev: np.ndarray, mu: float, gravity_norm: float,
               dt: float) -> np.ndarray:
    """Initial impulses from network outputs y and the previous dimensionless impulses prev:
    with s = y + prev, lambda_n = max(0, s_n) |g| dt / k_n and
    lambda_t = clip(s_t |g| dt / k_t, -mu lambda_n, mu lambda_n)."""
    y = y + prev
    gdt = gravity_norm * dt
    ln = np.maximum(0.0, y[..., 0]) * gdt / k[..., 0]
    b = mu * ln
    lt1 = np.clip(y[..., 1] * gdt / k[..., 1], -b, b)
    lt2 = np.clip(y[..., 2] * gdt / k[..., 2], -b, b)
    return np.stack([ln, lt1, lt2], axis=-1)
