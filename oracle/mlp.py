"""Plain FP64 multilayer perceptron -- TEST INFRASTRUCTURE ONLY.

The oracle of the surrogate network's HIP kernels (forward pass, mean
squared error, back-propagation, Adam).  The paper has no network; the
definitions followed here are the standard ones:

* GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (Hendrycks and Gimpel,
  "Gaussian Error Linear Units", 2016), derivative Phi(z) + z phi(z);
* Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015,
  Algorithm 1): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
* bfloat16: the upper 16 bits of an IEEE float32 after rounding the float32
  to nearest, ties to even, at bit 16.

Network: x -> (x - shift) * scale -> [Linear -> GELU] x depth -> Linear.
Linear layers hold W[out][in] and b[out]; y = h W^T + b.
Loss: mean over the batch and the outputs of (y - t)^2.

With ``emulate_bf16=True`` the stored quantities the kernels keep in
bfloat16 (the normalised input, the weights seen by the products, every
post-activation h, the output gradient dY and every pre-activation gradient
dZ) are rounded to bfloat16 at the same points, everything else stays FP64.
Matrix products use numpy's matmul (a library primitive).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (via float32, nearest-even) and return float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def layer_sizes(n_in: int, width: int, depth: int, n_out: int):
    """(out, in) of every Linear layer."""
    sizes = [(width, n_in)]
    sizes += [(width, width)] * (depth - 1)
    sizes += [(n_out, width)]
    return sizes


def unflatten(flat, n_in, width, depth, n_out):
    """Flat parameter vector (per layer: W row-major, then b) -> list of (W, b)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for (no, ni) in layer_sizes(n_in, width, depth, n_out):
        W = flat[o:o + no * ni].reshape(no, ni)
        o += no * ni
        b = flat[o:o + no]
        o += no
        out.append((W.copy(), b.copy()))
    assert o == flat.size, "parameter count does not match the shape"
    return out


def flatten(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def n_params(n_in, width, depth, n_out) -> int:
    return sum(no * ni + no for no, ni in layer_sizes(n_in, width, depth, n_out))


def forward(layers, x, shift, scale, emulate_bf16=False):
    """Returns (y, cache) with cache = (h_0 = normalised input, [z_l], [h_l])."""
    r = bf16_round if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    h = r((np.asarray(x, dtype=np.float64) - shift) * scale)
    hs, zs = [h], []
    for W, b in layers[:-1]:
        z = h @ r(W).T + b
        h = r(gelu(z))
        zs.append(z)
        hs.append(h)
    W, b = layers[-1]
    y = h @ r(W).T + b
    return y, (hs, zs)


def loss_and_grads(layers, x, t, shift, scale, emulate_bf16=False):
    """Mean squared error and its gradient with respect to every (W, b)."""
    r = bf16_round if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, (hs, zs) = forward(layers, x, shift, scale, emulate_bf16)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    loss = float(np.sum((y - t) ** 2) / n)
    dz = r(2.0 * (y - t) / n)               # gradient at the output (linear layer)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = hs[li]
        grads[li] = (dz.T @ h_in, dz.sum(axis=0))
        if li > 0:
            dh = dz @ r(W)
            dz = r(dh * gelu_grad(zs[li - 1]))
    return loss, y, grads


def adam_step(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
