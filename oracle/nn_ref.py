"""FP64 NumPy reference of the learned cell scorer (test infrastructure only).

The scorer is not part of the paper; it is this project's extension that
ranks orbit-grid cells from their coarse stamps so that the full stack runs
on promising cells only.  This module is the oracle its GPU kernels are
checked against: a plain forward pass, the hand-derived backward pass, the
binary cross-entropy loss and the Adam update, all in float64.  Gradients
are pinned by central finite differences in the tests.

Architecture (activations channels-last, weights in the GEMM layout
[K, N] with K = (ky * 3 + kx) * C_in + c_in for a 3x3 convolution):
  stamp 21x21x1 -> conv3x3 s1 (16) -> ReLU -> conv3x3 s2 (32) -> ReLU (11x11)
                -> conv3x3 s2 (32) -> ReLU (6x6) -> flatten 1152 -> FC 64 -> ReLU = h_img
  features 16   -> FC 64 -> ReLU = h_feat
  [h_img, h_feat] 128 -> FC 64 -> ReLU -> FC 1 = logit
All convolutions use zero padding 1.
"""
from __future__ import annotations

import numpy as np

STAMP = 21
NFEAT = 16

# (name, shape) of every parameter in the flat parameter vector, in order
LAYERS = [
    ("w1", (9 * 1, 16)), ("b1", (16,)),
    ("w2", (9 * 16, 32)), ("b2", (32,)),
    ("w3", (9 * 32, 32)), ("b3", (32,)),
    ("w4", (6 * 6 * 32, 64)), ("b4", (64,)),
    ("w5", (NFEAT, 64)), ("b5", (64,)),
    ("w6", (128, 64)), ("b6", (64,)),
    ("w7", (64, 1)), ("b7", (1,)),
]


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in LAYERS))


def unflatten(theta):
    out, off = {}, 0
    for name, shape in LAYERS:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[off:off + n], dtype=np.float64).reshape(shape)
        off += n
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in LAYERS])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in LAYERS:
        if name.startswith("w"):
            parts.append(rng.standard_normal(shape).ravel() * np.sqrt(2.0 / shape[0]))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)


def out_size(n, stride):
    return (n + 2 - 3) // stride + 1


def im2col(x, stride):
    """x: (B, H, W, C) -> (B, Ho, Wo, 9 C) with K index (ky * 3 + kx) * C + c."""
    B, H, W, C = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((B, H + 2, W + 2, C), dtype=x.dtype)
    xp[:, 1:H + 1, 1:W + 1, :] = x
    cols = np.empty((B, Ho, Wo, 9 * C), dtype=x.dtype)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            cols[..., (ky * 3 + kx) * C:(ky * 3 + kx + 1) * C] = patch
    return cols


def col2im(dcols, shape, stride):
    """Adjoint of im2col: scatter-add (B, Ho, Wo, 9 C) back to (B, H, W, C)."""
    B, H, W, C = shape
    Ho, Wo = dcols.shape[1], dcols.shape[2]
    dxp = np.zeros((B, H + 2, W + 2, C), dtype=dcols.dtype)
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :] += \
                dcols[..., (ky * 3 + kx) * C:(ky * 3 + kx + 1) * C]
    return dxp[:, 1:H + 1, 1:W + 1, :]


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, stamps, feats, keep=False):
    """stamps (B, 21, 21), feats (B, 16) -> logits (B,) [and the cache]."""
    p = unflatten(theta)
    B = stamps.shape[0]
    x0 = np.asarray(stamps, np.float64).reshape(B, STAMP, STAMP, 1)
    c1 = im2col(x0, 1)
    h1 = relu(c1 @ p["w1"] + p["b1"])                 # (B, 21, 21, 16)
    c2 = im2col(h1, 2)
    h2 = relu(c2 @ p["w2"] + p["b2"])                 # (B, 11, 11, 32)
    c3 = im2col(h2, 2)
    h3 = relu(c3 @ p["w3"] + p["b3"])                 # (B, 6, 6, 32)
    f3 = h3.reshape(B, -1)
    h4 = relu(f3 @ p["w4"] + p["b4"])
    f = np.asarray(feats, np.float64)
    h5 = relu(f @ p["w5"] + p["b5"])
    cat = np.concatenate([h4, h5], axis=1)
    h6 = relu(cat @ p["w6"] + p["b6"])
    z = (h6 @ p["w7"] + p["b7"])[:, 0]
    if keep:
        return z, dict(x0=x0, c1=c1, h1=h1, c2=c2, h2=h2, c3=c3, h3=h3, f3=f3, h4=h4, f=f, h5=h5, cat=cat, h6=h6)
    return z


def bce_with_logits(z, y):
    """Mean binary cross-entropy of logits z against labels y in {0, 1}."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_and_grad(theta, stamps, feats, labels):
    """(loss, dL/dtheta) by the chain rule, layer by layer."""
    p = unflatten(theta)
    z, c = forward(theta, stamps, feats, keep=True)
    B = z.shape[0]
    y = np.asarray(labels, np.float64)
    loss = bce_with_logits(z, y)
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B            # dL/dz
    g = {}
    g["w7"] = c["h6"].T @ dz[:, None]
    g["b7"] = np.array([dz.sum()])
    dh6 = dz[:, None] @ p["w7"].T
    d6 = dh6 * (c["h6"] > 0)
    g["w6"] = c["cat"].T @ d6
    g["b6"] = d6.sum(0)
    dcat = d6 @ p["w6"].T
    d4 = dcat[:, :64] * (c["h4"] > 0)
    d5 = dcat[:, 64:] * (c["h5"] > 0)
    g["w5"] = c["f"].T @ d5
    g["b5"] = d5.sum(0)
    g["w4"] = c["f3"].T @ d4
    g["b4"] = d4.sum(0)
    dh3 = (d4 @ p["w4"].T).reshape(c["h3"].shape)
    d3 = dh3 * (c["h3"] > 0)
    g["w3"] = c["c3"].reshape(-1, c["c3"].shape[-1]).T @ d3.reshape(-1, 32)
    g["b3"] = d3.reshape(-1, 32).sum(0)
    dh2 = col2im(d3 @ p["w3"].T, c["h2"].shape, 2)
    d2 = dh2 * (c["h2"] > 0)
    g["w2"] = c["c2"].reshape(-1, c["c2"].shape[-1]).T @ d2.reshape(-1, 32)
    g["b2"] = d2.reshape(-1, 32).sum(0)
    dh1 = col2im(d2 @ p["w2"].T, c["h1"].shape, 2)
    d1 = dh1 * (c["h1"] > 0)
    g["w1"] = c["c1"].reshape(-1, c["c1"].shape[-1]).T @ d1.reshape(-1, 16)
    g["b1"] = d1.reshape(-1, 16).sum(0)
    return loss, flatten(g)


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float64 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
