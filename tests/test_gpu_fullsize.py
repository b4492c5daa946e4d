"""GPU parity at the workloads' full sizes, through the C ABI.

References:
  * tests/golden/*.json, written by tests/golden/make_golden.py from the
    oracle alone: the 512 x 512 runs over their full 1e4 steps and 50/100-step
    prefixes of the 2048 x 2048 run (the full 5e4 steps would take the oracle
    about a day), each with the final observables and a seeded sample of
    final cells (the 64 densest cells plus 192 uniform ones);
  * for the full 2048 x 2048, 5e4-step FP32 run: the GPU FP64 run, which the
    prefix tests tie to the oracle on the same grid.
Bars: FP64 sampled cells within 1e-10 relative L2 and probabilities within
1e-12 of the oracle; FP32 probabilities within 1e-4 absolute and, each on
its own, within the FP32 error model of helpers.fp32_bars (a per-step
floor plus a relative part; 1 to 6 percent of the diffracted-order and
spin-flip probabilities of these runs).
"""
import json
import os

import numpy as np
import pytest

from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W
from helpers import check_fp32_probabilities

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def workload_of(rec) -> W.Workload:
    w = rec["workload"]
    return W.Workload(w["name"], W.GridSpec(**w["grid"]), W.BeamSpec(**w["beam"]), W.PacketSpec(**w["packet"]),
                      W.ObsSpec(**w["obs"]), dt=w["dt"], steps=w["steps"], t0=w["t0"], meta=w["meta"])


def run_gpu(wl, prec, steps, t0):
    print(f"[case] {wl.name} prec={prec} steps={steps} t0={t0}", flush=True)
    sim = qw.Sim(wl.grid, prec, beam=wl.beam)
    sim.init_packet(wl.packet)
    sim.step(steps, t0, wl.dt)
    obs = np.array(sim.observables(wl.obs))
    return sim, obs


def check_f64(rec):
    wl = workload_of(rec)
    sim, obs = run_gpu(wl, qw.QW_F64, rec["steps"], rec["t0"])
    ref_obs = np.array(rec["observables"])
    cells = rec["cells"]
    ref = np.array(rec["psi_re"]) + 1j * np.array(rec["psi_im"])
    psi = sim.state()
    got = np.array([psi[iy, ix] for iy, ix in cells])
    sim.close()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  sampled-cell rel L2 {err:.3e}, max |d obs| {np.max(np.abs(obs[1:] - ref_obs[1:])):.3e}, "
          f"norm diff {abs(obs[0] - ref_obs[0]):.3e}")
    assert err <= 1e-10
    assert abs(obs[0] - ref_obs[0]) <= 1e-11
    assert np.max(np.abs(obs[1:] - ref_obs[1:])) <= 1e-12


@pytest.mark.parametrize("name", ["large_prefix0", "large_prefix_field"])
def test_large_grid_prefix_f64_matches_oracle(name):
    check_f64(load(name))


@pytest.mark.parametrize("name", ["large_prefix0", "large_prefix_field"])
def test_large_grid_prefix_f32_matches_oracle(name):
    """FP32 at 2048^2 in the bench's launch sequence (graph replays plus
    direct launches) against the oracle's sampled cells and observables.
    Bar: the FP32 path's error grows linearly with the steps, a coherent
    drift of the norm (the nearest-rounded rotation constants lose about
    2e-7 per step, which the kinetic table's norm factor takes out on
    average) and of the phases, above the rounding noise sqrt(n log2 N)
    2^-24.  Measured without the norm factor: 9.6e-6 relative L2 after 100
    steps; the bar, 3e-7 n (3e-5 at 100 steps), keeps a factor three over
    that.  Probabilities (ratios to the current norm): helpers.fp32_bars."""
    rec = load(name)
    wl = workload_of(rec)
    sim, obs = run_gpu(wl, qw.QW_F32, rec["steps"], rec["t0"])
    ref_obs = np.array(rec["observables"])
    cells = rec["cells"]
    ref = np.array(rec["psi_re"]) + 1j * np.array(rec["psi_im"])
    psi = sim.state()
    got = np.array([psi[iy, ix] for iy, ix in cells])
    sim.close()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  FP32 sampled-cell rel L2 {err:.3e}")
    assert err <= 3e-7 * rec["steps"]
    check_fp32_probabilities(obs, ref_obs, wl.obs.n_max, rec["steps"], name)


@pytest.mark.parametrize("name", ["mid_w2", "mid_w4", "mid_w8"])
def test_mid_grid_full_run_f64_matches_oracle(name):
    check_f64(load(name))


@pytest.mark.parametrize("name", ["mid_w2", "mid_w4", "mid_w8"])
def test_mid_grid_full_run_f32_probabilities(name):
    """512^2, 1e4 steps, FP32 against the oracle's stored observables: every
    probability within helpers.fp32_bars (P_+1 = 8e-8 .. 1.4e-5 and
    P_flip = 1e-7 .. 9e-7 here; the bars are 3.6e-7 + 1e-3 P and
    1e-8 + 1e-2 P_flip), and within 1e-4."""
    rec = load(name)
    wl = workload_of(rec)
    sim, obs = run_gpu(wl, qw.QW_F32, rec["steps"], rec["t0"])
    sim.close()
    print(f"  norm drift {obs[0] - 1:.2e}")
    check_fp32_probabilities(obs, rec["observables"], wl.obs.n_max, rec["steps"], name)


def test_large_grid_full_run_f32_vs_f64():
    """The throughput workload (2048^2, 5e4 steps, the launch sequence bench.py
    times): FP32 against the GPU FP64 run, every probability within
    helpers.fp32_bars (P_+1 = 1.1e-4 with a bar of 1.9e-6, P_flip = 1.1e-6
    with a bar of 6e-8) and within 1e-4."""
    wl = W.large()
    _, o64 = run_gpu(wl, qw.QW_F64, wl.steps, 0.0)
    _, o32 = run_gpu(wl, qw.QW_F32, wl.steps, 0.0)
    print(f"  norm drift {o32[0] - 1:.2e}")
    check_fp32_probabilities(o32, o64, wl.obs.n_max, wl.steps, "2048^2 5e4 steps")
