"""Pins of the oracle's Dirac matrices, propagators and bispinors.

Sec. II.B: H = c alpha.(p + A) + beta c^2 in the standard representation
(Eq. 5), bispinors u^s (Eq. 9-10), energy E(p) (Eq. 11).  The propagators
are checked against scipy's matrix exponential of -i H tau, the
representation against the textbook Pauli/Dirac algebra, and the spinors
against the eigenvalue equation (Eq. 7).
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle

C = 137.036
I2 = np.eye(2)
I4 = np.eye(4)


def extracted_representation():
    """alpha_x, alpha_y, beta read back from the oracle's H0 at chosen momenta."""
    h00 = oracle.hamiltonian0(0.0, 0.0, C)
    beta = h00 / C ** 2
    ax = (oracle.hamiltonian0(1.0, 0.0, C) - h00) / C
    ay = (oracle.hamiltonian0(0.0, 1.0, C) - h00) / C
    return ax, ay, beta


def test_standard_representation():
    ax, ay, beta = extracted_representation()
    sz = np.diag([1.0, -1.0])
    assert np.allclose(beta, np.diag([1, 1, -1, -1]), atol=1e-14)
    sx = ax[0:2, 2:4]
    sy = ay[0:2, 2:4]
    # block-off-diagonal alpha_k = [[0, s_k], [s_k, 0]]
    for a, s in ((ax, sx), (ay, sy)):
        assert np.allclose(a[0:2, 0:2], 0) and np.allclose(a[2:4, 2:4], 0)
        assert np.allclose(a[2:4, 0:2], s)
    # Pauli algebra with sigma_z = diag(1,-1): s_x s_y = i s_z, s_x = [[0,1],[1,0]]
    assert np.allclose(sx, [[0, 1], [1, 0]])
    assert np.allclose(sx @ sy, 1j * sz, atol=1e-14)
    # Clifford relations {a_i, a_j} = 2 delta_ij, {a_i, beta} = 0, beta^2 = 1
    for a in (ax, ay):
        assert np.allclose(a @ a, I4) and np.allclose(a @ beta + beta @ a, 0)
        assert np.allclose(a, a.conj().T)
    assert np.allclose(ax @ ay + ay @ ax, 0)
    assert np.allclose(beta @ beta, I4)


@pytest.mark.parametrize("seed", range(6))
def test_kinetic_propagator_is_exp(seed):
    rng = np.random.default_rng(seed)
    px, py = rng.uniform(-200, 200, size=2)
    tau = rng.uniform(-1e-4, 1e-4)
    h = oracle.hamiltonian0(px, py, C)
    assert np.allclose(h, h.conj().T, atol=0)
    ev = np.linalg.eigvalsh(h)
    e = oracle.energy(px, py, C)
    assert np.allclose(np.sort(ev), [-e, -e, e, e], rtol=1e-13)
    assert abs(e - np.sqrt(C ** 4 + C ** 2 * (px * px + py * py))) <= 1e-13 * e
    k = oracle.kinetic_matrix(px, py, C, tau)
    ref = expm(-1j * h * tau)
    assert np.max(np.abs(k - ref)) <= 1e-13
    assert np.max(np.abs(k.conj().T @ k - I4)) <= 1e-14


@pytest.mark.parametrize("amag,tau", [(0.7, 5.7e-5), (3.0, 1e-3), (1e-9, 5.7e-5), (2e-5, 3e-5), (0.0, 5.7e-5),
                                      (0.5, -5.7e-5)])
def test_interaction_propagator_is_exp(amag, tau):
    ax_, ay_, _ = extracted_representation()
    rng = np.random.default_rng(int(amag * 1e3) + 5)
    ang = rng.uniform(0, 2 * np.pi)
    a = (amag * np.cos(ang), amag * np.sin(ang))
    m = ax_ * a[0] + ay_ * a[1]
    assert np.allclose(m @ m, amag ** 2 * I4, atol=1e-15)
    v = oracle.interaction_matrix(a[0], a[1], C, tau)
    ref = expm(-1j * C * m * tau)
    assert np.max(np.abs(v - ref)) <= 2e-15
    assert np.max(np.abs(v.conj().T @ v - I4)) <= 2e-15


def test_interaction_small_angle_branch_is_continuous():
    # theta = c |A| tau straddling the 1e-4 switch to the Taylor series
    tau = 5.7e-5
    for theta in (0.99e-4, 1.0e-4, 1.01e-4):
        amag = theta / (C * tau)
        v = oracle.interaction_matrix(amag, 0.0, C, tau)
        ax_, _, _ = extracted_representation()
        ref = expm(-1j * C * ax_ * amag * tau)
        assert np.max(np.abs(v - ref)) <= 1e-16 * 4


@pytest.mark.parametrize("seed", range(5))
def test_spinors(seed):
    rng = np.random.default_rng(100 + seed)
    px, py = rng.uniform(-300, 300, size=2)
    h = oracle.hamiltonian0(px, py, C)
    e = oracle.energy(px, py, C)
    up = oracle.spinor(px, py, C, +1)
    um = oracle.spinor(px, py, C, -1)
    for u in (up, um):
        assert abs(np.vdot(u, u) - 1) <= 1e-14
        assert np.max(np.abs(h @ u - e * u)) <= 1e-12 * e      # Eq. 7 eigenvalue relation
    assert abs(np.vdot(up, um)) <= 1e-14
    # upper two components proportional to chi^s (Eq. 9): chi^+ = (1,1), chi^- = (1,-1)
    assert abs(up[0] - up[1]) <= 1e-14 and abs(um[0] + um[1]) <= 1e-14


def test_spinors_at_rest_are_x_polarised():
    sx4 = np.kron(I2, np.array([[0, 1], [1, 0]]))   # Sigma_x = diag(sigma_x, sigma_x)
    up = oracle.spinor(0.0, 0.0, C, +1)
    um = oracle.spinor(0.0, 0.0, C, -1)
    assert np.allclose(sx4 @ up, up, atol=1e-15)
    assert np.allclose(sx4 @ um, -um, atol=1e-15)
    assert np.allclose(up, np.array([1, 1, 0, 0]) / np.sqrt(2), atol=1e-15)
