"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bars: FP64 state within 1e-10 relative L2 of the oracle (1e-12 for a few
steps), FP64 observables within 1e-12; FP32 runs within the FP32 rounding
bounds written per test.  Every input is seeded and synthetic.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W
from helpers import o_grid, o_beam, o_packet, o_obs, rel_l2, momenta

pytestmark = pytest.mark.gpu

F64, F32 = qw.QW_F64, qw.QW_F32


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def strong_beam(w0=1.0, a0=1.5):
    return W.BeamSpec(mode=W.BEAM_STANDING_PARAXIAL, a0=a0, w0=w0, ramp_periods=0.0, longitudinal=1)


def box(nx, ny, periods=8):
    L = periods * W.LAMBDA_L
    return W.GridSpec(nx=nx, ny=ny, x_min=-L / 2, y_min=-L / 2, lx=L, ly=L)


def print_case(**kw):
    print("[case] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("prec", [F64, F32])
def test_initial_packet_matches_oracle(prec):
    wl = W.small_parity()
    print_case(test="initial_packet", prec=prec, grid=wl.grid.nx)
    ref = oracle.init_packet(o_grid(wl.grid), o_packet(wl.packet))
    sim = qw.Sim(wl.grid, prec)
    sim.init_packet(wl.packet)
    got = sim.state()
    tol = 1e-13 if prec == F64 else 2e-6
    assert rel_l2(got, ref) <= tol
    assert abs(np.sum(np.abs(got) ** 2) - 1) <= (1e-13 if prec == F64 else 1e-5)


@pytest.mark.parametrize("prec", [F64, F32])
def test_observables_match_oracle(prec):
    wl = W.small_parity()
    print_case(test="observables", prec=prec)
    for psi in (oracle.init_packet(o_grid(wl.grid), o_packet(wl.packet)),
                W.random_state(wl.grid.ny, wl.grid.nx, seed=21)):
        ref = oracle.observables(o_grid(wl.grid), psi, o_obs(wl.obs))
        sim = qw.Sim(wl.grid, prec)
        sim.load(psi)
        if prec == F32:
            # compare against the oracle on the FP32-rounded state
            psi32 = psi.astype(np.complex64).astype(np.complex128)
            ref = oracle.observables(o_grid(wl.grid), psi32, o_obs(wl.obs))
        got = np.array(sim.observables(wl.obs))
        tol = 1e-13 if prec == F64 else 1e-6
        assert np.max(np.abs(got - ref)) <= tol, (got, ref)


@pytest.mark.parametrize("n_max,spin0,window,ref_shift", [(0, 1, 8, 0), (1, -1, 0, 3), (2, 1, 4, -5),
                                                          (16, -1, 8, 1)])
def test_observables_specs_match_oracle(n_max, spin0, window, ref_shift):
    # band windows from none to past every order the grid holds (n_max = 16:
    # the largest accepted, 3B + 3 = 102 sums, bands beyond |n| = 8 empty),
    # both spin references, window half-widths 0 .. k_L/dk / 2, shifted
    # reference columns; FP64 on a seeded random state of a 256 x 64 grid
    # (box 16 x 4 wavelengths)
    g = W.GridSpec(nx=256, ny=64, x_min=-4.0, y_min=-1.0, lx=8.0, ly=2.0)
    m = int(round(g.lx / W.LAMBDA_L))  # k_L / dk
    o = W.ObsSpec(band_ref_idx=-m + ref_shift, band_half_idx=m, window_idx=min(window, m // 2), n_max=n_max,
                  spin0=spin0)
    print_case(test="observables_specs", n_max=n_max, spin0=spin0, window=o.window_idx, ref=o.band_ref_idx)
    psi = W.random_state(g.ny, g.nx, seed=33)
    ref = oracle.observables(o_grid(g), psi, o_obs(o))
    sim = qw.Sim(g, F64)
    sim.load(psi)
    got = np.array(sim.observables(o))
    sim.close()
    assert got.shape == ref.shape == (3 * (2 * n_max + 1) + 3,)
    assert np.max(np.abs(got - ref)) <= 1e-13, float(np.max(np.abs(got - ref)))


# (2048, 32) and (4096, 32): long rows with one-row middle tiles whose line
# groups are dealt to one XCD (grids that are multiples of 8 x group size)
SIZES = [(8, 8), (16, 8), (8, 16), (32, 64), (64, 32), (128, 8), (8, 128), (256, 16), (16, 256),
         (512, 8), (8, 512), (1024, 8), (8, 1024), (2048, 8), (8, 2048), (4096, 8), (8, 4096), (2048, 32),
         (4096, 32)]


@pytest.mark.parametrize("nx,ny", SIZES)
def test_steps_all_sizes_f64(nx, ny):
    print_case(test="steps_f64", nx=nx, ny=ny)
    g = box(nx, ny)
    beam = strong_beam()
    psi0 = W.random_state(ny, nx, seed=nx * 7 + ny)
    t0 = 3.3 * W.T_L
    ref = oracle.step_n(o_grid(g), o_beam(beam), psi0, 3, t0, W.DT)
    sim = qw.Sim(g, F64, beam=beam)
    sim.load(psi0)
    sim.step(3, t0, W.DT)
    assert rel_l2(sim.state(), ref) <= 1e-12


@pytest.mark.parametrize("nx,ny", [(8, 8), (64, 32), (256, 16), (16, 256), (2048, 8), (8, 2048),
                                   (4096, 8), (8, 4096), (2048, 32), (4096, 32)])
def test_steps_all_sizes_f32(nx, ny):
    print_case(test="steps_f32", nx=nx, ny=ny)
    g = box(nx, ny)
    beam = strong_beam()
    psi0 = W.random_state(ny, nx, seed=nx * 5 + ny).astype(np.complex64).astype(np.complex128)
    t0 = 3.3 * W.T_L
    ref = oracle.step_n(o_grid(g), o_beam(beam), psi0, 3, t0, W.DT)
    sim = qw.Sim(g, F32, beam=beam)
    sim.load(psi0)
    sim.step(3, t0, W.DT)
    # a few ulp per butterfly stage: ~ (log2 nx + log2 ny) 6e-8 per transform, 12 transforms
    bound = 12 * (math.log2(nx) + math.log2(ny)) * 6e-8
    assert rel_l2(sim.state(), ref) <= bound


@pytest.mark.parametrize("prec", [F64, F32])
def test_small_parity_workload(prec):
    wl = W.small_parity()
    print_case(test="small_parity", prec=prec, steps=wl.steps)
    G = o_grid(wl.grid)
    ref = oracle.step_n(G, o_beam(wl.beam), oracle.init_packet(G, o_packet(wl.packet)), wl.steps, wl.t0, wl.dt)
    ref_obs = oracle.observables(G, ref, o_obs(wl.obs))
    sim = qw.Sim(wl.grid, prec, beam=wl.beam)
    sim.init_packet(wl.packet)
    sim.step(wl.steps, wl.t0, wl.dt)
    got_obs = np.array(sim.observables(wl.obs))
    if prec == F64:
        assert rel_l2(sim.state(), ref) <= 1e-10
        assert np.max(np.abs(got_obs - ref_obs)) <= 1e-12
    else:
        assert rel_l2(sim.state(), ref) <= 1e-4
        assert np.max(np.abs(got_obs[1:] - ref_obs[1:])) <= 1e-5
        assert abs(got_obs[0] - ref_obs[0]) <= 1e-4


def test_free_evolution_is_exact_phase_gpu():
    wl = W.small_parity()
    g = wl.grid
    print_case(test="free_evolution")
    sim = qw.Sim(g, F64, beam=W.BeamSpec(mode=W.BEAM_NONE))
    sim.init_packet(wl.packet)
    psi0 = sim.state()
    n = 200
    sim.step(n, 0.0, wl.dt)
    PX, PY = momenta(g)
    e = np.sqrt(g.c ** 4 + g.c ** 2 * (PX ** 2 + PY ** 2))
    exact = np.fft.ifft2(np.fft.fft2(psi0, axes=(0, 1)) * np.exp(-1j * e * n * wl.dt)[:, :, None], axes=(0, 1))
    assert rel_l2(sim.state(), exact) <= 1e-12


def test_uniform_field_matches_oracle():
    g = W.square_box(32, 8)
    print_case(test="uniform_field")
    beam = W.BeamSpec(mode=W.BEAM_UNIFORM, ux=0.5, uy=0.3)
    psi0 = oracle.init_packet(o_grid(g), o_packet(W.PacketSpec()))
    ref = oracle.step_n(o_grid(g), o_beam(beam), psi0, 64, 0.0, W.DT)
    sim = qw.Sim(g, F64, beam=beam)
    sim.load(psi0)
    sim.step(64, 0.0, W.DT)
    assert rel_l2(sim.state(), ref) <= 1e-12


def test_time_reversal_gpu():
    wl = W.small_parity()
    print_case(test="time_reversal")
    sim = qw.Sim(wl.grid, F64, beam=wl.beam)
    sim.init_packet(wl.packet)
    psi0 = sim.state()
    t0, n = 25 * W.T_L, 64
    sim.step(n, t0, wl.dt)
    assert rel_l2(sim.state(), psi0) > 1e-3
    sim.step(n, t0 + n * wl.dt, -wl.dt)
    assert rel_l2(sim.state(), psi0) <= 1e-12


def test_split_calls_agree():
    wl = W.small_parity()
    print_case(test="split_calls")
    a = qw.Sim(wl.grid, F64, beam=wl.beam)
    a.init_packet(wl.packet)
    b = qw.Sim(wl.grid, F64, beam=wl.beam)
    b.init_packet(wl.packet)
    a.step(50, 0.0, wl.dt)
    b.step(20, 0.0, wl.dt)
    b.step(30, 20 * wl.dt, wl.dt)
    assert rel_l2(b.state(), a.state()) <= 1e-13


@pytest.mark.parametrize("prec", [F64, F32])
def test_graph_replays_equal_direct_launches(prec):
    # 150 steps: two replays of the captured 64-step chunk plus 21 direct
    # steps, the middle passes of the two Dirac blocks as two chains on two
    # streams; with per-launch timing on, the loop launches every pass of
    # both blocks directly on the one stream.  Same arithmetic, same step
    # times: bitwise equal states.  Then a new beam (recapture) and a second
    # state array (another capture).
    wl = W.small_parity()
    print_case(test="graph_replays", prec=prec)
    a = qw.Sim(wl.grid, prec, beam=wl.beam)
    b = qw.Sim(wl.grid, prec, beam=wl.beam)
    a.init_packet(wl.packet)
    b.init_packet(wl.packet)
    qw.qw_kernel_timing(b.ctx, True)
    a.step(150, 0.0, wl.dt)
    b.step(150, 0.0, wl.dt)
    qw.qw_kernel_times(b.ctx, b.stream())
    assert np.array_equal(a.state(), b.state())
    beam2 = strong_beam(w0=1.5, a0=0.8)
    a.set_beam(beam2)
    b.set_beam(beam2)
    a.step(130, 150 * wl.dt, wl.dt)
    b.step(130, 150 * wl.dt, wl.dt)
    qw.qw_kernel_times(b.ctx, b.stream())
    assert np.array_equal(a.state(), b.state())
    other = a.psi.clone()
    a.psi, other = other, a.psi
    a.step(70, 280 * wl.dt, wl.dt)
    b.step(70, 280 * wl.dt, wl.dt)
    qw.qw_kernel_times(b.ctx, b.stream())
    assert np.array_equal(a.state(), b.state())
    a.close()
    b.close()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 129])
def test_block_chains_equal_single_stream(n):
    # the two-chain loop around the chunk boundaries (no middle step, one,
    # a chunk less one, a whole chunk, a chunk and one, two chunks and one)
    # equals the single-stream launches bit for bit
    wl = W.small_parity()
    print_case(test="block_chains", n=n)
    a = qw.Sim(wl.grid, F32, beam=wl.beam)
    b = qw.Sim(wl.grid, F32, beam=wl.beam)
    a.init_packet(wl.packet)
    b.init_packet(wl.packet)
    qw.qw_kernel_timing(b.ctx, True)
    a.step(n, 0.0, wl.dt)
    b.step(n, 0.0, wl.dt)
    qw.qw_kernel_times(b.ctx, b.stream())
    assert np.array_equal(a.state(), b.state())
    a.close()
    b.close()


def test_step_loop_captured_by_the_caller():
    # qw_step_n inside the caller's own graph capture (torch.cuda.graph):
    # plain launches are recorded; every replay, with eager work and
    # synchronisation in between, equals the same call made eagerly
    import torch
    wl = W.small_parity()
    print_case(test="caller_capture")
    a = qw.Sim(wl.grid, F32, beam=wl.beam)
    b = qw.Sim(wl.grid, F32, beam=wl.beam)
    for sim in (a, b):
        sim.init_packet(wl.packet)
        sim.step(1, 0.0, wl.dt)  # tables built outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        a.step(100, wl.dt, wl.dt)
    for r in range(3):
        g.replay()
        b.step(100, wl.dt, wl.dt)
        torch.cuda.synchronize()
        assert np.array_equal(a.state(), b.state()), f"replay {r}"
    del g
    a.close()
    b.close()


def test_n_zero_and_dt_zero():
    wl = W.small_parity()
    print_case(test="n0_dt0")
    sim = qw.Sim(wl.grid, F64, beam=wl.beam)
    sim.init_packet(wl.packet)
    psi0 = sim.state()
    sim.step(0, 0.0, wl.dt)
    assert np.array_equal(sim.state(), psi0)
    sim.step(5, 1.0 * W.T_L, 0.0)
    assert rel_l2(sim.state(), psi0) <= 1e-14


def test_block_decoupling_exact_gpu():
    wl = W.small_parity()
    print_case(test="block_decoupling")
    psi0 = W.random_state(wl.grid.ny, wl.grid.nx, seed=4)
    psi0[:, :, 1] = 0
    psi0[:, :, 2] = 0
    for prec in (F64, F32):
        sim = qw.Sim(wl.grid, prec, beam=wl.beam)
        sim.load(psi0)
        sim.step(10, 25 * W.T_L, wl.dt)
        psi = sim.state()
        assert np.all(psi[:, :, 1] == 0) and np.all(psi[:, :, 2] == 0)


def test_non_finite_state_reports_numeric_error():
    wl = W.small_parity()
    print_case(test="nan_state")
    psi0 = W.random_state(wl.grid.ny, wl.grid.nx, seed=5)
    psi0[3, 7, 2] = np.nan
    sim = qw.Sim(wl.grid, F64, beam=wl.beam)
    sim.load(psi0)
    rc, out = sim.observables(wl.obs, check=False)
    assert rc == qw.QW_E_NUMERIC
    assert "not finite" in qw.qw_last_error(sim.ctx)


def test_step_before_beam_is_a_state_error():
    wl = W.small_parity()
    sim = qw.Sim(wl.grid, F64)
    with pytest.raises(qw.QWError) as e:
        sim.step(1, 0.0, wl.dt)
    assert e.value.code == qw.QW_E_STATE


def test_kernel_timing_counts_launches():
    wl = W.small_parity()
    sim = qw.Sim(wl.grid, F32, beam=wl.beam)
    sim.init_packet(wl.packet)
    qw.qw_kernel_timing(sim.ctx, True)
    sim.step(10, 0.0, wl.dt)
    cnt_r, ms_r, cnt_c, ms_c = qw.qw_kernel_times(sim.ctx, sim.stream())
    assert cnt_r == 11 and cnt_c == 10 and ms_r > 0 and ms_c > 0
    qw.qw_kernel_timing(sim.ctx, False)
    sim.step(3, 0.0, wl.dt)
    assert qw.qw_kernel_times(sim.ctx, sim.stream())[0] == 0
