"""GPU parity of the full Gaussian-beam field (QW_BEAM_GAUSSIAN_FULL), the
moving box and the gauge shift (qw_set_frame), through the C ABI, against
the FP64 oracle.  Units follow the paper's showcase (hbar = m = 1 in atomic
units: hbar k_L = 0.1 m c, dt = 0.05 hbar/(m c^2)), on reduced grids.

Bars: FP64 state within 1e-10 relative L2, observables within 1e-12; FP32
state within 2e-5 relative L2 (float butterflies over log N passes and the
float propagators, a few hundred float roundings per value over these step
counts, with the phases formed in double).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W
from helpers import rel_l2

pytestmark = pytest.mark.gpu

C = W.C_AU
KL = 0.1 * C
LAM = 2 * math.pi / KL
DT = 0.05 / C ** 2


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def case(nx, ny, bx_lam, by_lam, y_min_lam, eps=0.1, a0=0.1 * C, longitudinal=1, p0y=0.3 * C, y0_lam=None,
         spin=1, sigma_lam=3.0):
    g = W.GridSpec(nx=nx, ny=ny, x_min=-bx_lam * LAM / 2, y_min=y_min_lam * LAM, lx=bx_lam * LAM, ly=by_lam * LAM)
    b = W.BeamSpec(mode=qw.QW_BEAM_GAUSSIAN_FULL, a0=a0, lambda_l=LAM, w0=1.0 / (KL * eps), ramp_periods=0.0,
                   longitudinal=longitudinal)
    y0 = (y_min_lam + by_lam / 2) * LAM if y0_lam is None else y0_lam * LAM
    p = W.PacketSpec(p0x=-KL, p0y=p0y, x0=0.0, y0=y0, sigma_x=sigma_lam * LAM, spin=spin)
    half = int(round(g.lx / LAM))
    o = W.ObsSpec(band_ref_idx=-half, band_half_idx=half, window_idx=half // 2, n_max=2, spin0=spin)
    return g, b, p, o


def o_all(g, b, p, o):
    G = oracle.Grid(g.nx, g.ny, g.x_min, g.y_min, g.lx, g.ly, g.c)
    B = oracle.Beam(b.mode, b.a0, b.lambda_l, b.w0, b.ramp_periods, b.longitudinal, b.ux, b.uy)
    P = oracle.Packet(p.p0x, p.p0y, p.x0, p.y0, p.sigma_x, p.spin)
    O = oracle.ObsSpec(o.band_ref_idx, o.band_half_idx, o.window_idx, o.n_max, o.spin0)
    return G, B, P, O


def run_both(g, b, p, o, prec, steps, vy=0.0, a_m=0.0, t0=0.0):
    print(f"[case] {g.nx}x{g.ny} prec={prec} steps={steps} vy={vy:.3g} a_m={a_m:.3g}", flush=True)
    G, B, P, O = o_all(g, b, p, o)
    F = oracle.Frame(vy=vy, a_m=a_m)
    ref = oracle.step_n(G, B, oracle.init_packet(G, P, frame=F), steps, t0, DT, frame=F)
    ref_obs = oracle.observables(G, ref, O, frame=F)
    sim = qw.Sim(g, prec, beam=b)
    sim.set_frame(vy, a_m)
    sim.init_packet(p)
    sim.step(steps, t0, DT)
    got = sim.state()
    obs = np.array(sim.observables(o))
    sim.close()
    return got, ref, obs, ref_obs


@pytest.mark.parametrize("longitudinal", [1, 0])
def test_full_beam_lab_frame_f64(longitudinal):
    g, b, p, o = case(128, 64, 16, 8, -4, longitudinal=longitudinal, y0_lam=0.0)
    got, ref, obs, ref_obs = run_both(g, b, p, o, qw.QW_F64, 60, t0=0.37 / (C * KL))
    err = rel_l2(got, ref)
    print(f"  rel L2 {err:.2e}, max |d obs| {np.max(np.abs(obs - ref_obs)):.2e}")
    assert err <= 1e-10
    assert np.max(np.abs(obs - ref_obs)) <= 1e-12


def test_full_beam_moving_box_and_gauge_shift_f64():
    # the showcase geometry scaled down: p_y = m c carried by the gauge shift
    # a_m = m c (grid momentum p_y = 0), the box following the packet at c/sqrt2
    g, b, p, o = case(256, 32, 40, 20, -14, eps=0.05, p0y=C, y0_lam=-4.0, sigma_lam=4.0)
    got, ref, obs, ref_obs = run_both(g, b, p, o, qw.QW_F64, 80, vy=C / math.sqrt(2), a_m=C)
    err = rel_l2(got, ref)
    print(f"  rel L2 {err:.2e}, max |d obs| {np.max(np.abs(obs - ref_obs)):.2e}")
    assert err <= 1e-10
    assert np.max(np.abs(obs - ref_obs)) <= 1e-12


def test_gauge_shift_with_paraxial_field_f64():
    g, b, p, o = case(128, 64, 16, 8, -4, y0_lam=0.0)
    b = W.BeamSpec(mode=qw.QW_BEAM_STANDING_PARAXIAL, a0=0.2 * C, lambda_l=LAM, w0=2 * LAM, ramp_periods=0.0)
    got, ref, obs, ref_obs = run_both(g, b, p, o, qw.QW_F64, 40, a_m=0.7 * C)
    assert rel_l2(got, ref) <= 1e-10
    assert np.max(np.abs(obs - ref_obs)) <= 1e-12


def test_full_beam_moving_box_f32():
    g, b, p, o = case(256, 32, 40, 20, -14, eps=0.05, p0y=C, y0_lam=-4.0, sigma_lam=4.0)
    got, ref, obs, ref_obs = run_both(g, b, p, o, qw.QW_F32, 80, vy=C / math.sqrt(2), a_m=C)
    err = rel_l2(got, ref)
    print(f"  FP32 rel L2 {err:.2e}, max |d obs| {np.max(np.abs(obs[1:] - ref_obs[1:])):.2e}")
    assert err <= 2e-5
    assert np.max(np.abs(obs[1:] - ref_obs[1:])) <= 1e-5


def test_moving_box_needs_a_per_cell_field():
    g, b, p, o = case(64, 64, 8, 8, -4)
    sim = qw.Sim(g, qw.QW_F64, beam=W.BeamSpec(mode=qw.QW_BEAM_STANDING_PARAXIAL, a0=1.0, lambda_l=LAM, w0=LAM))
    sim.set_frame(0.5 * C, 0.0)
    sim.init_packet(p)
    with pytest.raises(qw.QWError) as e:
        sim.step(3, 0.0, DT)
    assert e.value.code == qw.QW_E_STATE
    with pytest.raises(qw.QWError):
        sim.set_frame(1.5 * C, 0.0)
    sim.close()


def test_momentum_maps_match_oracle():
    g, b, p, o = case(64, 32, 8, 8, -4, y0_lam=0.0)
    a_m = 0.6 * C
    G, B, P, O = o_all(g, b, p, o)
    F = oracle.Frame(vy=0.0, a_m=a_m)
    ref = oracle.step_n(G, B, oracle.init_packet(G, P, frame=F), 15, 0.0, DT, frame=F)
    phi = oracle.dft2(ref)
    px = 2 * math.pi * np.fft.fftfreq(g.nx, d=g.lx / g.nx)
    py = 2 * math.pi * np.fft.fftfreq(g.ny, d=g.ly / g.ny)
    want = np.zeros((g.ny, g.nx, 3))
    for iy in range(g.ny):
        for ix in range(g.nx):
            f = phi[iy, ix]
            up = oracle.spinor(px[ix], py[iy] + a_m, C, 1)
            um = oracle.spinor(px[ix], py[iy] + a_m, C, -1)
            want[iy, ix] = (np.sum(np.abs(f) ** 2), abs(np.vdot(up, f)) ** 2, abs(np.vdot(um, f)) ** 2)
    print("[case] momentum maps 64x32", flush=True)
    sim = qw.Sim(g, qw.QW_F64, beam=b)
    sim.set_frame(0.0, a_m)
    sim.load(ref)
    got = sim.momentum_maps()
    sim.close()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(want)
