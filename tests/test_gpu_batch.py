"""GPU parity of the batched form (qw_batch_*), through the C ABI.

* FP64 batches of mixed, uneven grids against the FP64 oracle run on each
  instance alone: states within 1e-10 relative L2, observables within 1e-12,
  for the default schedules and for every schedule variant of every length;
* FP32 batches against the single-instance FP32 path, element by element:
  identical bits, with and without the captured step-loop graph and with
  persistent launches (the batched kernels run the same arithmetic);
* the step loop (middle steps in cooperative launches with grid-wide
  barriers between the phases): FP64 against the oracle as above, FP32
  identical bits to the launch-per-pass path, and a barrier wait past its
  limit (a zero limit set from the host; every workgroup still leaves the
  launch normally) reported by the next observables call;
* the autotuner leaves psi untouched and its choices keep FP64 parity;
* the full batching workload (96 instances of 256^2 / 512^2 / 1024^2 FP32,
  2e4 steps, autotuned) against the GPU FP64 single-instance runs of sampled
  instances -- which the oracle pins on smaller grids -- to 1e-4 in every
  probability.
"""
import numpy as np
import pytest

import oracle
from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W
from helpers import o_grid, o_beam, o_packet, o_obs, rel_l2, check_fp32_probabilities

pytestmark = pytest.mark.gpu

F64, F32 = qw.QW_F64, qw.QW_F32


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def print_case(**kw):
    print("[case] " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def grid(nx, ny, px, py):
    return W.GridSpec(nx=nx, ny=ny, x_min=-px * W.LAMBDA_L / 2, y_min=-py * W.LAMBDA_L / 2,
                      lx=px * W.LAMBDA_L, ly=py * W.LAMBDA_L)


def mixed_instances(sizes, seed=3, ramp=0.0):
    """Uneven grids with seeded field and packet parameters (strong fields, no
    ramp, so the interaction acts from the first step)."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (nx, ny, px, py) in enumerate(sizes):
        g = grid(nx, ny, px, py)
        b = W.BeamSpec(a0=float(rng.uniform(0.3, 1.5)), w0=float(rng.uniform(1.0, 3.0)), ramp_periods=ramp)
        p = W.PacketSpec(p0y=float(rng.uniform(0, 0.3)) * W.K_L, spin=1 if i % 2 == 0 else -1, sigma_x=1.0)
        out.append((g, b, p, W.obs_for(g, p, spin0=p.spin)))
    return out


MIXED = [(64, 64, 8, 8), (128, 64, 8, 4), (64, 128, 4, 8), (128, 128, 8, 8), (256, 256, 8, 8)]


def oracle_run(g, b, p, o, steps, t0, dt):
    psi = oracle.step_n(o_grid(g), o_beam(b), oracle.init_packet(o_grid(g), o_packet(p)), steps, t0, dt)
    return psi, np.array(oracle.observables(o_grid(g), psi, o_obs(o)))


def make_batch(cases, prec):
    bt = qw.Batch([(g, b) for g, b, _, _ in cases], prec)
    bt.init_packets([p for _, _, p, _ in cases])
    return bt


def loop_capacity(bt):
    """Step-loop workgroups that fit one CU (the device must allow cooperative launches)."""
    fit = bt.set_loop(-1)
    assert fit >= 1, "no step-loop workgroup fits a CU, or no cooperative launches"
    return fit


@pytest.mark.parametrize("graph_steps,loop", [(0, 0), (8, 0), (8, 2), (0, 1), (8, qw.QW_LOOP_INSTANCE)])
def test_batch_f64_matches_oracle(graph_steps, loop):
    cases = mixed_instances(MIXED)
    steps, t0, dt = 37, 0.25 * W.T_L, W.DT
    print_case(test="batch_f64", graph_steps=graph_steps, loop=loop, steps=steps)
    bt = make_batch(cases, F64)
    bt.set_launch(0, 0, graph_steps)
    if loop:
        bt.set_loop(loop if loop == qw.QW_LOOP_INSTANCE else min(loop, loop_capacity(bt)))
    bt.step(steps, t0, dt)
    obs = bt.observables([o for *_, o in cases])
    for i, (g, b, p, o) in enumerate(cases):
        ref, ref_obs = oracle_run(g, b, p, o, steps, t0, dt)
        err = rel_l2(bt.state(i), ref)
        d = np.max(np.abs(np.array(obs[i]) - ref_obs))
        print(f"  instance {i} {g.nx}x{g.ny}: rel L2 {err:.2e}, max |d obs| {d:.2e}")
        assert err <= 1e-10
        assert d <= 1e-12
    bt.close()


def test_batch_f64_every_schedule_variant_matches_oracle():
    sizes = [(64, 64, 8, 8), (128, 128, 8, 8), (256, 256, 8, 8), (512, 64, 16, 2), (1024, 64, 32, 2),
             (64, 512, 2, 16), (64, 1024, 2, 32)]
    cases = mixed_instances(sizes, seed=5)
    steps, dt = 9, W.DT
    refs = [oracle_run(g, b, p, o, steps, 0.0, dt)[0] for g, b, p, o in cases]
    for v in range(4):
        print_case(test="batch_variants_f64", variant=v)
        bt = make_batch(cases, F64)
        for lg in range(6, 11):
            nv = len([u for u in range(4) if bt.schedule(lg, u)])
            for pass_ in (0, 1):
                bt.set_schedule(lg, pass_, min(v, nv - 1))
        bt.set_launch(0, 0, 4)
        bt.step(steps, 0.0, dt)
        for i in range(len(cases)):
            err = rel_l2(bt.state(i), refs[i])
            assert err <= 1e-10, (v, i, err)
        bt.close()


def single_run(g, b, p, prec, steps, t0, dt):
    sim = qw.Sim(g, prec, beam=b)
    sim.init_packet(p)
    sim.step(steps, t0, dt)
    out = sim.state()
    sim.close()
    return out


@pytest.mark.parametrize("launch", [(0, 0, 0), (0, 0, 16), (2, 2, 16), (1, 4, 5)])
def test_batch_f32_is_bitwise_the_single_instance_path(launch):
    sizes = [(256, 256, 8, 8), (512, 512, 16, 16), (1024, 1024, 32, 32), (64, 256, 2, 8), (2048, 64, 64, 2)]
    cases = mixed_instances(sizes, seed=7, ramp=2.0)
    steps, dt = 41, W.DT
    print_case(test="batch_f32_bitwise", launch=launch, steps=steps)
    bt = make_batch(cases, F32)
    bt.set_launch(*launch)
    bt.step(steps, 0.0, dt)
    for i, (g, b, p, _) in enumerate(cases):
        ref = single_run(g, b, p, F32, steps, 0.0, dt)
        got = bt.state(i)
        assert np.array_equal(got, ref), (i, float(np.max(np.abs(got - ref))))
    bt.close()


@pytest.mark.parametrize("wg,graph_steps", [(1, 16), (2, 0), (2, 5), (qw.QW_LOOP_INSTANCE, 16),
                                             (qw.QW_LOOP_INSTANCE, 0)])
def test_step_loop_is_bitwise_the_launch_per_pass_path(wg, graph_steps):
    """FP32 uneven grids (64 to 2048 points per line): the middle steps in
    step-loop launches of graph_steps steps (64 when 0), with grid-wide
    barriers or one workgroup per instance, against the same batch advanced
    one launch per pass: identical bits, and no barrier wait ran past its
    limit (observables would raise)."""
    sizes = [(256, 256, 8, 8), (512, 512, 16, 16), (1024, 1024, 32, 32), (64, 256, 2, 8), (2048, 64, 64, 2)]
    cases = mixed_instances(sizes, seed=7, ramp=2.0)
    steps = 41
    print_case(test="step_loop_f32_bitwise", wg=wg, graph_steps=graph_steps, steps=steps)
    ref = make_batch(cases, F32)
    ref.set_launch(0, 0, 0)
    ref.step(steps, 0.0, W.DT)
    bt = make_batch(cases, F32)
    bt.set_launch(0, 0, graph_steps)
    bt.set_loop(wg if wg == qw.QW_LOOP_INSTANCE else min(wg, loop_capacity(bt)))
    bt.step(steps, 0.0, W.DT)
    bt.observables([o for *_, o in cases])
    for i in range(len(cases)):
        got, exp = bt.state(i), ref.state(i)
        assert np.array_equal(got, exp), (i, float(np.max(np.abs(got - exp))))
    bt.close()
    ref.close()


def test_step_loop_wait_limit_is_reported_once():
    """A barrier wait limit of zero, set from the host, ends the step-loop
    launch early (every workgroup leaves normally): the next observables
    call reports it; the report clears it, and the loop with the default
    limit then reproduces the launch-per-pass result bit for bit."""
    cases = mixed_instances(MIXED[:3], seed=5)
    specs = [o for *_, o in cases]
    print_case(test="step_loop_wait_limit")
    bt = make_batch(cases, F32)
    bt.set_launch(0, 0, 0)
    bt.set_loop(1, wait_limit_s=1e-12)
    bt.step(10, 0.0, W.DT)
    with pytest.raises(qw.QWError, match="step-loop barrier"):
        bt.observables(specs)
    bt.set_loop(1)
    bt.init_packets([p for _, _, p, _ in cases])
    bt.step(10, 0.0, W.DT)
    bt.observables(specs)
    ref = make_batch(cases, F32)
    ref.set_launch(0, 0, 0)
    ref.step(10, 0.0, W.DT)
    for i in range(len(cases)):
        assert np.array_equal(bt.state(i), ref.state(i)), i
    bt.close()
    ref.close()


def test_batch_step_loop_captured_by_the_caller():
    # qw_batch_step_n inside the caller's own graph capture (torch.cuda.graph):
    # plain launches are recorded even where the batch would replay its own
    # graph (20 steps, chunks of 8); every replay equals the eager call
    import torch
    cases = mixed_instances(MIXED[:3], seed=17)
    print_case(test="batch_caller_capture")
    a = make_batch(cases, F32)
    b = make_batch(cases, F32)
    for bt in (a, b):
        bt.set_launch(0, 0, 8)
        bt.step(1, 0.0, W.DT)  # descriptors and kinetic tables set up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        a.step(20, W.DT, W.DT)
    for r in range(3):
        g.replay()
        b.step(20, W.DT, W.DT)
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert np.array_equal(a.state(i), b.state(i)), (r, i)
    del g
    a.close()
    b.close()


def test_batch_runs_continue_across_calls():
    """Two calls of n1 and n2 steps from t0 and t0 + n1 dt equal the oracle's
    n1 + n2 steps up to the merged half steps' rounding."""
    cases = mixed_instances(MIXED[:3], seed=11)
    dt = W.DT
    print_case(test="batch_continue")
    bt = make_batch(cases, F64)
    bt.set_launch(0, 0, 4)
    bt.step(13, 0.0, dt)
    bt.step(10, 13 * dt, dt)
    for i, (g, b, p, o) in enumerate(cases):
        ref, _ = oracle_run(g, b, p, o, 23, 0.0, dt)
        assert rel_l2(bt.state(i), ref) <= 1e-10
    bt.close()


def test_batch_autotune_leaves_psi_and_keeps_parity():
    cases = mixed_instances(MIXED, seed=13)
    print_case(test="batch_autotune_f64")
    bt = make_batch(cases, F64)
    before = bt.psi.clone()
    rows = bt.autotune(W.DT, reps=3)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(before, bt.psi)
    kinds = {int(r[0]) for r in rows}
    assert kinds == {0, 1, 2, 3, 4}
    # MIXED holds a 256^2 instance (64 tiles per step): no instance-loop candidate
    assert {int(r[1]) for r in rows if int(r[0]) == 4} == set(range(loop_capacity(bt) + 1))
    assert all(r[3] > 0 for r in rows)
    steps = 20
    bt.step(steps, 0.0, W.DT)
    for i, (g, b, p, o) in enumerate(cases):
        ref, _ = oracle_run(g, b, p, o, steps, 0.0, W.DT)
        assert rel_l2(bt.state(i), ref) <= 1e-10
    bt.close()


def test_autotune_times_the_instance_loop_on_small_grids():
    """Six 64^2 FP32 instances (4 tiles per step each): the instance loop is
    a middle-step candidate; on the default schedules, whichever middle-step
    path the autotuner keeps advances the batch to the same bits as the
    launch-per-pass path."""
    cases = mixed_instances([(64, 64, 8, 8)] * 6, seed=19)
    print_case(test="autotune_instance_loop")
    bt = make_batch(cases, F32)
    rows = bt.autotune(W.DT, reps=2)
    assert qw.QW_LOOP_INSTANCE in {int(r[1]) for r in rows if int(r[0]) == 4}
    for pass_ in (0, 1):  # default schedules (the tuned ones round differently); the loop choice stays
        bt.set_schedule(6, pass_, 0)
    bt.init_packets([p for _, _, p, _ in cases])
    bt.step(70, 0.0, W.DT)
    bt.observables([o for *_, o in cases])
    ref = make_batch(cases, F32)
    ref.set_launch(0, 0, 0)
    ref.step(70, 0.0, W.DT)
    for i in range(len(cases)):
        assert np.array_equal(bt.state(i), ref.state(i)), i
    bt.close()
    ref.close()


def test_batch_errors_are_reported():
    cases = mixed_instances(MIXED[:2])
    bt = make_batch(cases, F64)
    with pytest.raises(qw.QWError):
        bt.set_schedule(6, 0, 3)  # 64 has two FP64 variants
    with pytest.raises(qw.QWError):
        bt.set_launch(-1, 0, 0)
    with pytest.raises(qw.QWError):
        bt.set_loop(1, wait_limit_s=61.0)
    with pytest.raises(qw.QWError):
        bt.set_loop(bt.set_loop(-1) + 1)
    with pytest.raises(qw.QWError):
        bt.step(-1, 0.0, W.DT)
    o = W.ObsSpec(band_ref_idx=0, band_half_idx=4, window_idx=4)
    with pytest.raises(qw.QWError):
        bt.observables([o, o])
    bt.close()


@pytest.mark.timeout(900)
def test_full_batching_workload_f32_vs_f64():
    """96 instances, N in {256, 512, 1024}, 2e4 steps, FP32, autotuned,
    graph-captured: every instance's probabilities against the same batch
    run in FP64 (whose batched kernels match the oracle to 1e-10 above),
    each within helpers.fp32_bars and 1e-4."""
    wls = W.batch_instances(seed=0)
    steps = wls[0].steps
    print_case(test="batch_full_f32", instances=len(wls), steps=steps)
    bt = qw.Batch([(w.grid, w.beam) for w in wls], F32)
    bt.init_packets([w.packet for w in wls])
    bt.autotune(W.DT, reps=5)
    bt.init_packets([w.packet for w in wls])
    bt.step(steps, 0.0, W.DT)
    obs = bt.observables([w.obs for w in wls])
    bt.close()
    nb = 2 * wls[0].obs.n_max + 1
    for i, w in enumerate(wls):
        o = obs[i]
        assert abs(o[0] - 1.0) <= 1e-2, (i, o[0])          # FP32 norm drift
        assert -1e-6 <= o[1 + 3 * nb] <= 1.0                # P_flip
        assert sum(o[1:1 + nb]) <= 1.0 + 1e-9
    print_case(test="batch_full_f64", instances=len(wls), steps=steps)
    bt = qw.Batch([(w.grid, w.beam) for w in wls], F64)
    bt.init_packets([w.packet for w in wls])
    bt.step(steps, 0.0, W.DT)
    ref = bt.observables([w.obs for w in wls])
    bt.close()
    for i, w in enumerate(wls):
        check_fp32_probabilities(obs[i], ref[i], w.obs.n_max, steps, f"instance {i} ({w.grid.nx}^2)")
