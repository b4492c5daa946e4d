"""Pins of the oracle's FFT (the discretised Fourier pair, Sec. II.C Eq. 14).

Independent references: an O(N^4) brute-force DFT written as the definition,
numpy's FFT, Parseval's identity and inverse-after-forward = identity.
"""
import numpy as np
import pytest

import oracle


def brute_dft2(a, sign=-1):
    """Direct double sum X[ky,kx] = sum_{y,x} a[y,x] exp(sign 2 pi i (ky y/ny + kx x/nx))."""
    ny, nx = a.shape
    out = np.zeros_like(a, dtype=np.complex128)
    for ky in range(ny):
        for kx in range(nx):
            s = 0j
            for y in range(ny):
                for x in range(nx):
                    s += a[y, x] * np.exp(sign * 2j * np.pi * (ky * y / ny + kx * x / nx))
            out[ky, kx] = s
    return out


@pytest.mark.parametrize("ny,nx", [(8, 8), (16, 8), (8, 16)])
def test_dft2_matches_bruteforce(ny, nx):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((ny, nx, 4)) + 1j * rng.standard_normal((ny, nx, 4))
    got = oracle.dft2(a, -1)
    for c in range(4):
        ref = brute_dft2(a[:, :, c])
        assert np.max(np.abs(got[:, :, c] - ref)) <= 1e-13 * np.max(np.abs(ref))
    back = oracle.dft2(a, +1)
    for c in range(4):
        ref = brute_dft2(a[:, :, c], +1) / (nx * ny)
        assert np.max(np.abs(back[:, :, c] - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [1, 2, 4, 8, 32, 256, 4096])
def test_fft1d_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = oracle.fft1d(x, -1)
    ref = np.fft.fft(x)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.sqrt(np.log2(max(n, 2))) * np.linalg.norm(ref) + 1e-300
    inv = oracle.fft1d(x, +1)
    assert np.linalg.norm(inv - n * np.fft.ifft(x)) <= 1e-14 * np.sqrt(np.log2(max(n, 2))) * np.linalg.norm(inv)


def test_fft1d_rejects_non_power_of_two():
    with pytest.raises(RuntimeError):
        oracle.fft1d(np.zeros(12, dtype=np.complex128))


def test_dft2_parseval_and_identity():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((32, 64, 4)) + 1j * rng.standard_normal((32, 64, 4))
    f = oracle.dft2(a, -1)
    assert abs(np.sum(np.abs(f) ** 2) / (32 * 64) - np.sum(np.abs(a) ** 2)) <= 1e-13 * np.sum(np.abs(a) ** 2)
    back = oracle.dft2(f, +1)
    assert np.linalg.norm(back - a) <= 1e-14 * np.linalg.norm(a)
    ref = np.fft.fft2(a, axes=(0, 1))
    assert np.linalg.norm(f - ref) <= 1e-14 * np.linalg.norm(ref)


def test_dft2_thread_count_invariant():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((64, 32, 4)) + 1j * rng.standard_normal((64, 32, 4))
    n0 = oracle.get_threads()
    try:
        oracle.set_threads(1)
        f1 = oracle.dft2(a, -1)
        oracle.set_threads(4)
        f4 = oracle.dft2(a, -1)
    finally:
        oracle.set_threads(n0)
    assert np.array_equal(f1, f4)
