"""Lifetime of contexts and captured step loops, through the C ABI.

A caller may change the field, the launch shape or the state array, or
destroy a context, right after a qw_step_n / qw_batch_step_n whose graph
replays are still running on its stream.  The library then waits for the
last replay before it releases the executable graph.  These tests make such
calls back to back with no synchronisation in between and check every result
bit for bit against the same sequence run with a synchronisation after each
call (the arithmetic is identical, only the waiting differs).
"""
import numpy as np
import pytest

from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W

pytestmark = pytest.mark.gpu

F32 = qw.QW_F32


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def sync():
    import torch
    torch.cuda.synchronize()


def case(n=256, a0=0.8):
    g = W.square_box(n, n // 32)
    b = W.BeamSpec(a0=a0, w0=2.0 * W.LAMBDA_L, ramp_periods=0.0)
    p = W.PacketSpec(sigma_x=1.0)
    return g, b, p


def test_recapture_after_beam_change_with_replays_in_flight():
    """step (graph) -> new beam -> step (recaptured graph), unsynchronised vs synchronised."""
    g, b, p = case()
    b2 = W.BeamSpec(a0=0.3, w0=3.0 * W.LAMBDA_L, ramp_periods=0.0)
    out = []
    for wait in (False, True):
        print(f"[case] recapture wait={wait}", flush=True)
        sim = qw.Sim(g, F32, beam=b)
        sim.init_packet(p)
        sim.step(200, 0.0, W.DT)
        if wait:
            sync()
        sim.set_beam(b2)
        sim.step(200, 200 * W.DT, W.DT)
        out.append(sim.state())
        sim.close()
    assert np.array_equal(out[0], out[1])


def test_contexts_created_stepped_destroyed_back_to_back():
    """Six contexts, each destroyed right after its graph-replayed steps were enqueued."""
    g, b, p = case(n=128)
    kept = []
    for i in range(6):
        print(f"[case] back-to-back context {i}", flush=True)
        sim = qw.Sim(g, F32, beam=W.BeamSpec(a0=0.2 + 0.1 * i, w0=2.0 * W.LAMBDA_L, ramp_periods=0.0))
        sim.init_packet(p)
        sim.step(150, 0.0, W.DT)
        kept.append((sim.psi, sim.ws))  # the caller's memory outlives the context
        sim.close()  # no synchronisation before the destroy
    sync()
    for i, (psi, _) in enumerate(kept):
        ref = qw.Sim(g, F32, beam=W.BeamSpec(a0=0.2 + 0.1 * i, w0=2.0 * W.LAMBDA_L, ramp_periods=0.0))
        ref.init_packet(p)
        ref.step(150, 0.0, W.DT)
        sync()
        got = psi.detach().cpu().numpy()
        exp = ref.psi.detach().cpu().numpy()
        ref.close()
        assert np.array_equal(got, exp), i


def test_batch_relaunch_and_destroy_with_replays_in_flight():
    """Batched: step (graph) -> new graph chunk length -> step, then destroy, unsynchronised vs synchronised."""
    cases = [case(n=128, a0=0.5), case(n=256, a0=0.9)]
    out = []
    for wait in (False, True):
        print(f"[case] batch relaunch wait={wait}", flush=True)
        bt = qw.Batch([(g, b) for g, b, _ in cases], F32)
        bt.init_packets([p for _, _, p in cases])
        bt.set_launch(0, 0, 16)
        bt.step(100, 0.0, W.DT)
        if wait:
            sync()
        bt.set_launch(0, 0, 8)
        bt.step(100, 100 * W.DT, W.DT)
        views = [bt.view(i) for i in range(len(cases))]
        keep = bt.psi
        bt.close()  # right after the second step_n
        sync()
        out.append([v.detach().cpu().numpy().copy() for v in views])
        del keep
    for a, c in zip(out[0], out[1]):
        assert np.array_equal(a, c)
