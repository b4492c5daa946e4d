"""Pins of the oracle's split-operator propagation (Sec. II.D, Eq. 15) and of
the initial packet (Sec. II.C, Eq. 12-14) and observables (Sec. III.B, Eq. 18-19).

References that do not come from the oracle itself:
  * free evolution is exactly exp(-i E(p) t) on positive-energy states (Eq. 7, 11);
  * a uniform A has the closed-form solution exp(-i H0(p + A) t), computed here
    with scipy's expm, which the symmetric split approaches at second order;
  * unitarity (norm), time reversibility of the symmetric split, the block
    structure of the Dirac matrices at p_z = A_z = 0, mirror symmetry x -> -x;
  * the packet's position-space width and mean momentum (Eq. 12).
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from paper_2307_01571_amd import workloads as W
from helpers import o_grid, o_beam, o_packet, o_obs, rel_l2, momenta


def test_free_evolution_is_exact_phase():
    wl = W.small_parity()
    g, G = wl.grid, o_grid(wl.grid)
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    none = oracle.Beam(mode=oracle.BEAM_NONE)
    n = 200
    psi = oracle.step_n(G, none, psi0, n, 0.0, wl.dt)
    PX, PY = momenta(g)
    e = np.sqrt(g.c ** 4 + g.c ** 2 * (PX ** 2 + PY ** 2))        # Eq. 11
    phi = np.fft.fft2(psi0, axes=(0, 1)) * np.exp(-1j * e * n * wl.dt)[:, :, None]
    exact = np.fft.ifft2(phi, axes=(0, 1))
    assert rel_l2(psi, exact) <= 1e-12


def test_uniform_field_converges_at_second_order():
    g = W.square_box(32, 8)
    G = o_grid(g)
    psi0 = oracle.init_packet(G, o_packet(W.PacketSpec()))
    ux, uy = 0.5, 0.3
    beam = oracle.Beam(mode=oracle.BEAM_UNIFORM, ux=ux, uy=uy)
    T = 2 * W.T_L
    # exact: exp(-i H0(p + A) T) per momentum, with H0 from the textbook matrices
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]])
    z = np.zeros((2, 2))
    ax = np.block([[z, sx], [sx, z]])
    ay = np.block([[z, sy], [sy, z]])
    beta = np.diag([1.0, 1.0, -1.0, -1.0])
    phi0 = np.fft.fft2(psi0, axes=(0, 1))
    PX, PY = momenta(g)
    phiT = np.empty_like(phi0)
    for iy in range(g.ny):
        for ix in range(g.nx):
            h = g.c * (ax * (PX[iy, ix] + ux) + ay * (PY[iy, ix] + uy)) + beta * g.c ** 2
            phiT[iy, ix] = expm(-1j * h * T) @ phi0[iy, ix]
    exact = np.fft.ifft2(phiT, axes=(0, 1))
    errs = [rel_l2(oracle.step_n(G, beam, psi0, n, 0.0, T / n), exact) for n in (256, 512, 1024)]
    for a, b in zip(errs, errs[1:]):
        assert 3.6 <= a / b <= 4.4
    assert errs[-1] < 5e-5


def test_strang_order_with_standing_wave():
    g = W.square_box(32, 8)
    G = o_grid(g)
    psi0 = oracle.init_packet(G, o_packet(W.PacketSpec()))
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=2.0, lambda_l=W.LAMBDA_L, w0=1.0,
                       ramp_periods=0.0, longitudinal=1)
    T = W.T_L
    ref = oracle.step_n(G, beam, psi0, 64 * 64, 0.0, T / (64 * 64))
    errs = [rel_l2(oracle.step_n(G, beam, psi0, n, 0.0, T / n), ref) for n in (64, 128, 256)]
    for a, b in zip(errs, errs[1:]):
        assert 3.6 <= a / b <= 4.4


def test_norm_conservation_small_parity_case():
    wl = W.small_parity()
    G = o_grid(wl.grid)
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    assert abs(np.sum(np.abs(psi0) ** 2) - 1) <= 1e-14
    psi = oracle.step_n(G, o_beam(wl.beam), psi0, wl.steps, wl.t0, wl.dt)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) <= 1e-12


def test_time_reversal():
    wl = W.small_parity()
    G, B = o_grid(wl.grid), o_beam(wl.beam)
    # start after the ramp so the field is at full strength
    t0 = 25 * W.T_L
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    n = 64
    fwd = oracle.step_n(G, B, psi0, n, t0, wl.dt)
    assert rel_l2(fwd, psi0) > 1e-3
    back = oracle.step_n(G, B, fwd, n, t0 + n * wl.dt, -wl.dt)
    assert rel_l2(back, psi0) <= 1e-12


def test_block_decoupling_is_exact():
    wl = W.small_parity()
    g, G, B = wl.grid, o_grid(wl.grid), o_beam(wl.beam)
    psi0 = W.random_state(g.ny, g.nx, seed=4)
    psi0[:, :, 1] = 0
    psi0[:, :, 2] = 0
    psi = oracle.step_n(G, B, psi0, 10, 25 * W.T_L, wl.dt)
    assert np.all(psi[:, :, 1] == 0) and np.all(psi[:, :, 2] == 0)
    assert np.sum(np.abs(psi[:, :, 0]) ** 2) > 0.1


def test_mirror_symmetry_at_normal_incidence():
    """x -> -x with M = beta Sigma_x maps H to itself (A_x odd, A_y even in x) and
    u^+(p_x, p_y) to u^+(-p_x, p_y), so P_n^s = P_{-n}^s.  The grid keeps the
    symmetry except at the Nyquist column, which this box leaves empty."""
    length = 8 * W.LAMBDA_L
    g = W.GridSpec(nx=128, ny=32, x_min=-length / 2, y_min=-length / 2, lx=length, ly=length)
    pk = W.PacketSpec(p0x=0.0, p0y=0.1 * W.K_L)
    G = o_grid(g)
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=4.0, lambda_l=W.LAMBDA_L, w0=1.0,
                       ramp_periods=0.0, longitudinal=1)
    psi = oracle.step_n(G, beam, oracle.init_packet(G, o_packet(pk)), 150, 0.0, W.DT)
    spec = oracle.ObsSpec(band_ref_idx=0, band_half_idx=8, window_idx=4, n_max=2, spin0=1)
    o = oracle.unpack_observables(oracle.observables(G, psi, spec), 2)
    assert o["P"][3] > 1e-6 and o["Pm"][3] > 1e-12     # the field did diffract and flip
    for key in ("P", "Pp", "Pm"):
        v = o[key]
        assert np.all(np.abs(v - v[::-1]) <= 1e-15 + 1e-9 * np.abs(v)), (key, v)


def test_initial_packet_observables():
    wl = W.small_parity()
    G = o_grid(wl.grid)
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    o = oracle.unpack_observables(oracle.observables(G, psi0, o_obs(wl.obs)), wl.obs.n_max)
    assert abs(o["norm"] - 1) <= 1e-14
    assert abs(o["P"][2] - 1) <= 1e-14 and abs(o["Pp"][2] - 1) <= 1e-13
    assert abs(o["P_flip"]) <= 1e-14 and abs(o["P_neg"]) <= 1e-13
    assert np.all(np.abs(np.delete(o["P"], 2)) <= 1e-14)


def test_initial_packet_shape():
    """Width and mean momentum of the packet on a fine momentum grid (Eq. 12)."""
    g = W.square_box(256, 64)                    # dk = kL/64, sigma_p = 1.7 dk
    pk = W.PacketSpec(p0x=-W.K_L, p0y=0.1 * W.K_L, x0=1.0, y0=-2.0, sigma_x=1.5)
    psi0 = oracle.init_packet(o_grid(g), o_packet(pk))
    phi = np.fft.fft2(psi0, axes=(0, 1))
    w = np.sum(np.abs(phi) ** 2, axis=2)
    PX, PY = momenta(g)
    assert abs(np.sum(w * PX) / np.sum(w) - pk.p0x) <= 1e-9 * W.K_L
    assert abs(np.sum(w * PY) / np.sum(w) - pk.p0y) <= 1e-9 * W.K_L
    # position density: mean r0, standard deviation sigma_x per axis
    dens = np.sum(np.abs(psi0) ** 2, axis=2)
    x = g.x_min + g.lx * np.arange(g.nx) / g.nx
    y = g.y_min + g.ly * np.arange(g.ny) / g.ny
    X, Y = np.meshgrid(x, y)
    mx, my = np.sum(dens * X), np.sum(dens * Y)
    assert abs(mx - pk.x0) < 1e-3 and abs(my - pk.y0) < 1e-3
    sx = math.sqrt(np.sum(dens * (X - mx) ** 2))
    sy = math.sqrt(np.sum(dens * (Y - my) ** 2))
    # the relativistic spinor factor changes the width by O((p/c)^2) ~ 1e-2
    assert abs(sx / pk.sigma_x - 1) < 2e-2 and abs(sy / pk.sigma_x - 1) < 2e-2


def test_band_index_definition():
    """Closed windows |k - (r + 2 n m)| <= h enumerated from the definition."""
    for r, m, h in ((-16, 16, 8), (0, 8, 4), (5, 3, 2), (-64, 64, 32), (3, 4, 0), (0, 5, 4)):
        for k in range(-5 * m + r, 5 * m + r):
            n_def = [n for n in range(-6, 7) if abs(k - (r + 2 * n * m)) <= h]
            want = n_def[0] if n_def else oracle.NO_BAND
            assert oracle.band_index(k, r, m, h) == want


def test_observables_thread_invariant_and_spin_complete():
    wl = W.small_parity()
    G = o_grid(wl.grid)
    psi = W.random_state(wl.grid.ny, wl.grid.nx, seed=9)
    n0 = oracle.get_threads()
    try:
        oracle.set_threads(1)
        a = oracle.observables(G, psi, o_obs(wl.obs))
        oracle.set_threads(3)
        b = oracle.observables(G, psi, o_obs(wl.obs))
    finally:
        oracle.set_threads(n0)
    assert np.array_equal(a, b)
    o = oracle.unpack_observables(a, wl.obs.n_max)
    # a random state has about half its weight in negative-energy states
    assert 0.3 < o["P_neg"] < 0.7
    # P_n^+ + P_n^- <= P_n  (projection onto the positive-energy subspace)
    assert np.all(o["Pp"] + o["Pm"] <= o["P"] + 1e-15)
    # each window holds (2h+1) of the nx columns: about that share of a white state;
    # on this 64-point grid only the windows of orders 0 and +1 lie inside the grid
    frac = (2 * wl.obs.window_idx + 1) / wl.grid.nx
    assert np.all(np.abs(o["P"][2:4] / frac - 1) < 0.3)
    assert o["P"][0] == 0 and o["P"][1] == 0 and o["P"][4] == 0


def test_weak_field_two_photon_scaling():
    """Bragg diffraction into n = +1 is a two-photon process: P_1 ~ A0^4 at weak field
    (the windows leave out the one-photon sidebands at p0 +- kL, which go as A0^2)."""
    wl = W.small_parity()
    G = o_grid(wl.grid)
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    vals = []
    for a0 in (0.02, 0.04):
        b = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=a0, lambda_l=W.LAMBDA_L, w0=wl.beam.w0,
                        ramp_periods=0.0, longitudinal=1)
        psi = oracle.step_n(G, b, psi0, 200, 0.0, wl.dt)
        vals.append(oracle.unpack_observables(oracle.observables(G, psi, o_obs(wl.obs)), 2)["P"][3])
    slope = math.log(vals[1] / vals[0]) / math.log(2.0)
    assert abs(slope - 4) <= 0.2, vals
