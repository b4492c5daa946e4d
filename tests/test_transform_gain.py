"""The FP32 transforms' norm-gain model (qw_transform_gain), host only.

In float every rotation constant and twiddle of the transforms is the
nearest float of its cos and of its sin, so its squared magnitude falls
a little short of 1 and every transform loses a little norm, the same from
step to step.  The library models the mean loss per transform and divides
the kinetic table by it.  Here the model is checked against the exact
squared Frobenius norm of the transform's linear map, built by running the
kernels' transform structure (Stockham passes; radix 16 as 4 x 4 and radix
8 as 2 x 4 with the rotation constants between the two stages) in float64
arithmetic with the float-rounded constants, on every unit vector: for
inputs with independent entries, E|F'x|^2 / E|Fx|^2 = |F'|_F^2 / (N N).
The same structure with exact constants is numpy's FFT, which pins it.
"""
import numpy as np
import pytest

from paper_2307_01571_amd import qw

F32, F64 = qw.QW_F32, qw.QW_F64

PLANS_F32 = {8: (8,), 16: (16,), 32: (8, 4), 64: (16, 4), 128: (16, 8), 256: (16, 16), 512: (16, 8, 4),
             1024: (16, 16, 4), 2048: (16, 16, 8)}


def rot(angle, f32):
    c, s = np.cos(angle), np.sin(angle)
    if f32:
        c, s = float(np.float32(c)), float(np.float32(s))
    return complex(c, s)


def w16(j, f32, inv=False):
    j %= 16
    if j % 4 == 0:
        return [1, -1j, -1, 1j][j // 4] if not inv else [1, 1j, -1, -1j][j // 4]
    z = rot(2 * np.pi * j / 16, f32)
    return z if inv else z.conjugate()


def radix(x, R, f32):
    """Radix-R DFT over axis 0 of x (R rows), in the kernels' decomposition."""
    W4 = np.exp(-2j * np.pi * np.outer(np.arange(4), np.arange(4)) / 4)
    if R == 2:
        return np.stack([x[0] + x[1], x[0] - x[1]])
    if R == 4:
        return W4 @ x if x.ndim == 1 else np.tensordot(W4, x, axes=(1, 0))
    if R == 8:   # n = q + 2 l, k = s + 4 u
        y = np.stack([np.tensordot(W4, x[q::2], axes=(1, 0)) for q in range(2)])  # y[q, s]
        for s in range(4):
            y[1, s] = y[1, s] * w16(2 * s, f32)
        out = np.empty_like(x)
        for s in range(4):
            out[s] = y[0, s] + y[1, s]
            out[s + 4] = y[0, s] - y[1, s]
        return out
    if R == 16:  # n = q + 4 l, k = s + 4 u
        y = np.stack([np.tensordot(W4, x[q::4], axes=(1, 0)) for q in range(4)])  # y[q, s]
        for q in range(4):
            for s in range(4):
                y[q, s] = y[q, s] * w16(q * s, f32)
        out = np.empty_like(x)
        for s in range(4):
            z = np.tensordot(W4, y[:, s], axes=(1, 0))  # over q
            for u in range(4):
                out[s + 4 * u] = z[u]
        return out
    raise ValueError(R)


def stockham(x, radices, f32, split_rotations=False):
    """Forward transform of the columns of x (N rows) by Stockham passes.
    split_rotations: the radix-8/16 rotation constants exact (the library
    built with QW_F32_SPLIT_ROTATIONS=1 holds them as hi + lo pairs)."""
    inner = f32 and not split_rotations
    N = x.shape[0]
    ns = 1
    for R in radices:
        nb = N // R
        j = np.arange(nb)
        jm = j % ns
        inp = np.stack([x[j + r * nb] for r in range(R)])  # (R, nb, cols)
        if ns > 1:
            for r in range(R):
                tw = np.array([rot(-2 * np.pi * m * r / (ns * R), f32) for m in range(ns)])
                inp[r] = inp[r] * tw[jm][:, None]
        out = radix(inp, R, inner)
        y = np.empty_like(x)
        for r in range(R):
            y[(j // ns) * ns * R + jm + r * ns] = out[r]
        x = y
        ns *= R
    return x


def exact_gain(n, radices, split):
    F = stockham(np.eye(n, dtype=complex), radices, f32=True, split_rotations=split)
    return float(np.sum(np.abs(F) ** 2)) / (n * n)


_SPLIT = None


def split_build() -> bool:
    """Whether the library was built with split rotation constants: its
    modelled gain for 256 points is the exact map's for one of the two
    constant sets (asserted in test_the_build_matches_one_constant_set)."""
    global _SPLIT
    if _SPLIT is None:
        g = qw.qw_transform_gain(256, F32)
        _SPLIT = abs(g - exact_gain(256, PLANS_F32[256], True)) < abs(g - exact_gain(256, PLANS_F32[256], False))
    return _SPLIT


def test_the_build_matches_one_constant_set():
    g = qw.qw_transform_gain(256, F32)
    plain, split = exact_gain(256, PLANS_F32[256], False), exact_gain(256, PLANS_F32[256], True)
    assert abs(plain - split) > 1e-8                      # the two are told apart
    assert min(abs(g - plain), abs(g - split)) <= 2e-12


@pytest.mark.parametrize("n", [32, 256, 1024])
def test_structure_is_the_dft_with_exact_constants(n):
    F = stockham(np.eye(n, dtype=complex), PLANS_F32[n], f32=False)
    assert np.allclose(F, np.fft.fft(np.eye(n), axis=0), atol=1e-11)


@pytest.mark.parametrize("n", sorted(PLANS_F32))
def test_single_plan_gain_matches_the_exact_map(n):
    exact = exact_gain(n, PLANS_F32[n], split_build())
    got = qw.qw_transform_gain(n, F32)
    print(f"n {n}: gain - 1 = {got - 1:+.4e} (exact map {exact - 1:+.4e})")
    assert abs(got - exact) <= 2e-12
    assert -1e-7 < got - 1 <= 0         # a loss, of a few 1e-8 (none with exact rotations and no twiddles)
    assert qw.qw_transform_gain(n, F64) == 1.0


@pytest.mark.parametrize("lg,v", [(6, 1), (7, 2), (9, 1), (9, 3), (10, 1), (10, 2), (10, 3)])
def test_batch_variant_gain_matches_the_exact_map(lg, v):
    # the batched schedule variants of these lengths (qw_batch_schedule lists them per batch)
    n = 1 << lg
    radices = {(6, 1): (4, 16), (7, 2): (4, 4, 8), (9, 1): (8, 8, 8), (9, 3): (16, 16, 2), (10, 1): (16, 8, 8),
               (10, 2): (4, 16, 16), (10, 3): (8, 8, 16)}[(lg, v)]
    exact = exact_gain(n, radices, split_build())
    assert abs(qw.qw_transform_gain(n, F32, v) - exact) <= 2e-12


def test_gain_rejects_bad_lengths():
    for n in (0, 3, 1 << 13):
        with pytest.raises(qw.QWError):
            qw.qw_transform_gain(n, F32)
    with pytest.raises(qw.QWError):
        qw.qw_transform_gain(1024, F32, 9)


def test_per_bin_gains_of_the_float_transform_pair():
    """The round trip of one row pass in free flight (inverse, then forward
    transform, 1/N) as an exact linear map with the float-rounded constants:
    nearly diagonal, with a gain per frequency bin whose spread (a few 1e-8
    per step) the mean-gain factor in K does not remove.  Bins -80 and +80
    of a 2048-point row over 80 wavelengths (p_x = -k_L and +k_L) lose
    amounts per step that differ by about 6e-8."""
    n = 2048
    F = stockham(np.eye(n, dtype=complex), PLANS_F32[n], f32=True)
    M = F @ np.conj(F) / n
    g2 = np.abs(np.diag(M)) ** 2
    off = float(np.sum(np.abs(M - np.diag(np.diag(M))) ** 2)) / n
    mean = float(np.mean(g2))
    print(f"mean |g|^2 - 1 = {mean - 1:+.3e}, spread (std) {np.std(g2):.3e}; "
          f"bin -80: {g2[-80] - 1:+.3e}, bin +80: {g2[80] - 1:+.3e}; off-diagonal {off:.2e} per row")
    if not split_build():
        assert abs((mean - 1) - 2 * (qw.qw_transform_gain(n, F32) - 1)) < 1e-9   # two transforms per round trip
    assert 1e-8 < np.std(g2) < 1e-7
    assert 3e-8 < abs(g2[80] - g2[-80]) < 1e-7
    assert off < 1e-13



def test_a_lo_part_survives_only_before_the_rounding():
    """The split rotation constants (hi + lo floats): the lo product must
    enter the sum before the hi product is rounded.  With float values
    emulated exactly in double (a float product is exact there), rounding
    a c_hi + a c_lo once gives a c on average; adding a c_lo to the rounded
    a c_hi changes it only where the lo product reaches half a unit in the
    last place (near the top of a binade), so most of the constant's
    rounding stays, the same at every call."""
    rng = np.random.default_rng(7)
    a = rng.uniform(0.5, 2.0, 200_000).astype(np.float32).astype(np.float64)
    c = np.cos(2 * np.pi / 16)
    hi = float(np.float32(c))
    lo = float(np.float32(c - hi))
    assert lo != 0.0 and abs(lo) < 2.0 ** -24 * abs(hi)
    f32 = lambda x: x.astype(np.float32).astype(np.float64)
    before = f32(a * hi + a * lo)          # one rounding: fma(a, hi, a lo)
    after = f32(f32(a * hi) + a * lo)      # fma(a, lo, fl(a hi))
    hi_only = f32(a * hi)
    rel = lambda y: float(np.mean((y - a * c) / (a * c)))
    assert abs(rel(before)) < 2e-10                          # unbiased
    assert abs(rel(hi_only) - (hi - c) / c) < 2e-10          # the constant's rounding, coherent
    assert np.mean(after != hi_only) < 0.1                   # the lo part is mostly lost
    assert abs(rel(after)) > 0.8 * abs(rel(hi_only))
