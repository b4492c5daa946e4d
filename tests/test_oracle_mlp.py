"""Pins of the FP64 MLP oracle (the reference of the surrogate network's kernels).

Checked against what the definitions and the mathematics fix, not against
the oracle itself: tabulated values and an exact identity of GELU, central
differences of the loss for every parameter block, the closed form of the
first Adam steps, torch's own bfloat16 conversion, and a per-neuron loop
for the forward pass.
"""
import math

import numpy as np
import pytest

from oracle import mlp as M
from paper_2307_01571_amd import workloads as W


def test_gelu_values_and_identity():
    # Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208 (normal table)
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(M.gelu(2.0) - 2 * 0.9772498680518208) < 1e-15
    assert M.gelu(0.0) == 0.0
    x = np.linspace(-6, 6, 97)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.max(np.abs(M.gelu(x) - M.gelu(-x) - x)) < 1e-14
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-16


def test_gelu_grad_matches_central_differences():
    x = np.linspace(-5, 5, 41)
    h = 1e-5
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - M.gelu_grad(x))) < 1e-9


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 8, 2000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(v), ref)
    # ties go to even
    assert M.bf16_round(1.0 + 2 ** -8) == 1.0
    assert M.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def small_net(seed=1, n_in=5, width=16, depth=3, n_out=6, B=7):
    rng = np.random.default_rng(seed)
    layers = M.unflatten(W.mlp_init_params(seed, n_in, width, depth, n_out), n_in, width, depth, n_out)
    layers = [(Wt, rng.standard_normal(Wt.shape[0]) * 0.1) for Wt, _ in layers]
    x = rng.standard_normal((B, n_in))
    t = rng.standard_normal((B, n_out)) * 0.3
    shift = rng.standard_normal(n_in) * 0.1
    scale = 1.0 + rng.random(n_in)
    return layers, x, t, shift, scale


def test_gradients_match_central_differences():
    layers, x, t, shift, scale = small_net()
    loss, _, grads = M.loss_and_grads(layers, x, t, shift, scale)
    h = 1e-6
    for li, (Wt, b) in enumerate(layers):
        for which, arr in ((0, Wt), (1, b)):
            flat = arr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 13)):
                old = flat[idx]
                flat[idx] = old + h
                lp = M.loss_and_grads(layers, x, t, shift, scale)[0]
                flat[idx] = old - h
                lm = M.loss_and_grads(layers, x, t, shift, scale)[0]
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][which].reshape(-1)[idx]
                assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (li, which, idx, fd, an)


def test_forward_matches_per_neuron_loop():
    layers, x, t, shift, scale = small_net(seed=4, width=8, depth=2, B=3)
    y, _ = M.forward(layers, x, shift, scale)
    for s in range(x.shape[0]):
        h = [(x[s, i] - shift[i]) * scale[i] for i in range(x.shape[1])]
        for li, (Wt, b) in enumerate(layers):
            out = []
            for o in range(Wt.shape[0]):
                z = b[o] + sum(Wt[o, i] * h[i] for i in range(len(h)))
                out.append(z if li == len(layers) - 1 else 0.5 * z * (1 + math.erf(z / math.sqrt(2))))
            h = out
        assert np.max(np.abs(np.array(h) - y[s])) < 1e-13


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr = 1e-3
    p1, m, v = M.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    # bias-corrected first step: m^ = g, v^ = g^2  =>  dp = -lr g / (|g| + eps)
    assert np.max(np.abs(p1 - (p - lr * g / (np.abs(g) + 1e-8)))) < 1e-15
    g2 = rng.standard_normal(50)
    p2, _, _ = M.adam_step(p1, g2, m, v, 2, lr)
    mh = (0.9 * 0.1 * g + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g * g + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    assert np.max(np.abs(p2 - (p1 - lr * mh / (np.sqrt(vh) + 1e-8)))) < 1e-15


def test_emulated_bf16_stays_close_to_fp64():
    layers, x, t, shift, scale = small_net(seed=3, width=64, depth=4, B=32)
    l64, y64, g64 = M.loss_and_grads(layers, x, t, shift, scale)
    lb, yb, gb = M.loss_and_grads(layers, x, t, shift, scale, emulate_bf16=True)
    assert np.max(np.abs(yb - y64)) <= 0.05 * np.max(np.abs(y64))
    for (a, _), (b, _) in zip(g64, gb):
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(a)


def test_flatten_roundtrip_and_count():
    n = M.n_params(5, 256, 4, 6)
    assert n == 5 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 6 + 6
    p = W.mlp_init_params(0, 5, 256, 4, 6)
    assert p.size == n
    assert np.array_equal(M.flatten(M.unflatten(p, 5, 256, 4, 6)), p)
