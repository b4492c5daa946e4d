"""Pins of the oracle's full Gaussian-beam field (Sec. II.A, Eq. 1-4), the
co-moving box and the constant gauge shift A_m (Sec. II.D), checked against
what the formulas and the mathematics fix:

* closed forms of the two-beam sum at the focus and on the beam axis
  (sum-to-product of the d = +1 and d = -1 terms, Gouy phase included);
* parity in x and y of each component;
* the paraxial limit x << x_R: the separately pinned paraxial field with the
  amplitude doubled and the time shifted by a quarter period;
* the 2D divergence vanishes like eps^3 as the beam divergence eps -> 0 (a
  wrong sign or a dropped Gouy/curvature term leaves an O(eps) or O(eps^2)
  remainder);
* a box moving by one grid cell per step is the lab run translated by one
  cell per step, exactly;
* a gauge shift A_m of a whole number of momentum cells is a translation of
  the momentum-space state by those cells, exactly, field or no field.
"""
import math

import numpy as np
import pytest

import oracle

C = 137.036
KL = 0.1 * C          # paper units: hbar k_L = 0.1 m c
LAM = 2 * math.pi / KL
OM = C * KL


def full_beam(eps, a0=1.0, longitudinal=1, ramp=0.0):
    return oracle.Beam(mode=oracle.BEAM_GAUSSIAN_FULL, a0=a0, lambda_l=LAM, w0=1.0 / (KL * eps),
                       ramp_periods=ramp, longitudinal=longitudinal)


def test_full_beam_at_focus_and_on_axis():
    eps = 0.05
    b = full_beam(eps, a0=0.7)
    w0 = 1 / (KL * eps)
    xr = KL * w0 * w0 / 2
    for t in (0.0, 0.13 / OM, 1.7 / OM, 4.0 / OM):
        ax, ay = oracle.beam_eval(b, C, 0.0, 0.0, t)
        assert abs(ay - (-2 * 0.7 * math.sin(OM * t))) < 1e-14 and ax == 0.0
        for x in (0.37 * LAM, 3.1 * LAM, xr, -2.5 * xr):
            w = w0 * math.sqrt(1 + x * x / (xr * xr))
            ax, ay = oracle.beam_eval(b, C, x, 0.0, t)
            ref = -2 * 0.7 * (w0 / w) * math.sin(OM * t) * math.cos(KL * x - math.atan(x / xr))
            assert abs(ay - ref) < 1e-13 and abs(ax) < 1e-15


def test_full_beam_parities():
    b = full_beam(0.1)
    rng = np.random.default_rng(0)
    for _ in range(50):
        x, y = rng.uniform(-30 * LAM, 30 * LAM), rng.uniform(-10 * LAM, 10 * LAM)
        t = rng.uniform(0, 10 / OM)
        ax, ay = oracle.beam_eval(b, C, x, y, t)
        for sx, sy in ((-1, 1), (1, -1), (-1, -1)):
            bx, by = oracle.beam_eval(b, C, sx * x, sy * y, t)
            assert abs(by - ay) <= 1e-12 * (1 + abs(ay))          # A_y even in x and y
            assert abs(bx - sx * sy * ax) <= 1e-12 * (1 + abs(ax))  # A_x odd in x and in y


def test_full_beam_reduces_to_the_paraxial_field():
    eps = 1e-3
    w0 = 1 / (KL * eps)
    full = full_beam(eps, a0=0.5)
    par = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=1.0, lambda_l=LAM, w0=w0, ramp_periods=0.0,
                      longitudinal=1)
    quarter = 0.25 * (2 * math.pi / OM)
    worst_y = worst_x = 0.0
    for x in np.linspace(-5 / KL, 5 / KL, 11):
        for y in np.linspace(-2 * w0, 2 * w0, 11):
            for t in (0.1 / OM, 1.3 / OM):
                fx, fy = oracle.beam_eval(full, C, x, y, t)
                px, py = oracle.beam_eval(par, C, x, y, t + quarter)
                worst_y = max(worst_y, abs(fy - py))
                worst_x = max(worst_x, abs(fx - px))
    assert worst_y <= 1e-4 * 1.0       # scale of A_y: 2 A0 = 1
    assert worst_x <= 1e-4 * eps       # scale of A_x: O(eps)


def divergence_ratio(eps):
    b = full_beam(eps)
    w0 = 1 / (KL * eps)
    h = 1e-4 / KL
    t = 0.3 / OM
    worst = amax = 0.0
    for x in np.linspace(-20 * LAM, 20 * LAM, 9):
        for y in np.linspace(-2 * w0, 2 * w0, 9):
            axp, _ = oracle.beam_eval(b, C, x + h, y, t)
            axm, _ = oracle.beam_eval(b, C, x - h, y, t)
            _, ayp = oracle.beam_eval(b, C, x, y + h, t)
            _, aym = oracle.beam_eval(b, C, x, y - h, t)
            worst = max(worst, abs((axp - axm) / (2 * h) + (ayp - aym) / (2 * h)))
            amax = max(amax, abs(oracle.beam_eval(b, C, x, y, t)[1]))
    return worst / (KL * amax)


def test_full_beam_divergence_vanishes_like_eps_cubed():
    r = [divergence_ratio(e) for e in (0.04, 0.02, 0.01)]
    assert r[0] < 1e-3
    for a, b in zip(r, r[1:]):
        assert 7.0 < a / b < 9.0, r


def small_grid(n=64, periods=16):
    L = periods * 0.5
    return oracle.Grid(n, n, -L / 2, -L / 2, L, L, C)


def test_moving_box_is_the_translated_lab_run():
    g = small_grid()
    dy = g.ly / g.ny
    vy = C / math.sqrt(2)
    dt = dy / vy                      # the box moves one cell per step
    # a field that vanishes at the box edges in y: the moving box sees the
    # field beyond its edge, the fixed periodic box its periodic image
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=2.0, lambda_l=0.5, w0=0.5, ramp_periods=0.0)
    pk = oracle.Packet(-2 * math.pi / 0.5, 30.0, 0.0, 0.0, 1.0, 1)
    psi0 = oracle.init_packet(g, pk)
    n = 7
    lab = oracle.step_n(g, beam, psi0, n, 0.0, dt)
    box = oracle.step_n(g, beam, psi0, n, 0.0, dt, frame=oracle.Frame(vy=vy, a_m=0.0))
    # box point iy stands for the lab point iy + n
    assert np.max(np.abs(box - np.roll(lab, -n, axis=0))) <= 1e-12


@pytest.mark.parametrize("with_field", [False, True])
def test_gauge_shift_is_a_momentum_translation(with_field):
    g = small_grid()
    dk = 2 * math.pi / g.ly
    m = 5
    am = m * dk
    beam = (oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=1.5, lambda_l=0.5, w0=1.0, ramp_periods=0.0)
            if with_field else oracle.Beam(mode=oracle.BEAM_NONE))
    pk = oracle.Packet(-2 * math.pi / 0.5, 8 * dk, 0.0, 0.0, 1.0, -1)
    f = oracle.Frame(vy=0.0, a_m=am)
    a = oracle.step_n(g, beam, oracle.init_packet(g, pk, frame=f), 9, 0.0, 2e-4, frame=f)
    b = oracle.step_n(g, beam, oracle.init_packet(g, pk), 9, 0.0, 2e-4)
    fa, fb = oracle.dft2(a), np.roll(oracle.dft2(b), -m, axis=0)
    # canonical p in the shifted gauge is kinetic p - a_m: phi_a[ky] = phi_b[ky + m], up to the
    # constant phase exp(-i a_m (y_min - y0)) the two packets' position-space phases differ by
    ph = np.vdot(fb, fa) / abs(np.vdot(fb, fa))
    assert abs(ph - np.exp(-1j * am * (g.y_min - pk.y0))) < 1e-12
    assert np.max(np.abs(fa - ph * fb)) <= 1e-12 * np.max(np.abs(fb))
    o = oracle.ObsSpec(band_ref_idx=-4, band_half_idx=4, window_idx=2, n_max=2, spin0=-1)
    oa = oracle.observables(g, a, o, frame=f)
    ob = oracle.observables(g, b, o)
    assert np.max(np.abs(oa - ob)) <= 1e-12


def test_packet_in_a_gauge_shift_sits_at_kinetic_p0():
    g = small_grid(128, 32)
    dk = 2 * math.pi / g.ly
    f = oracle.Frame(vy=0.0, a_m=C)
    pk = oracle.Packet(-4 * math.pi, C + 3 * dk, 0.0, 0.0, 3.0, 1)
    phi = oracle.dft2(oracle.init_packet(g, pk, frame=f))
    w = np.sum(np.abs(phi) ** 2, axis=2)
    py = 2 * math.pi * np.fft.fftfreq(g.ny, d=g.ly / g.ny)
    mean_py = float(np.sum(w * py[:, None]) / np.sum(w))
    assert abs(mean_py + f.a_m - pk.p0y) < 1e-6 * C
    o = oracle.ObsSpec(band_ref_idx=-32, band_half_idx=32, window_idx=16, n_max=2, spin0=1)
    out = oracle.unpack_observables(oracle.observables(g, oracle.init_packet(g, pk, frame=f), o, frame=f), 2)
    # the packet is built from positive-energy, spin-up spinors of the kinetic momentum
    assert abs(out["Pp"][2] - 1) < 1e-12 and out["P_flip"] < 1e-12 and abs(out["P_neg"]) < 1e-12
