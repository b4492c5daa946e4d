"""The learned form end to end on the GPU: solver data from batched runs,
the ensemble trained by the library's kernels, and the fallback policy.

* every generated sample is exactly the single-instance solver's answer for
  its parameters and time (same kernels, same reduction order: 1e-12);
* a network trained on held-in runs predicts held-out runs, its queries are
  more than 100 times faster than one solve, and every query the policy
  sends to the solver returns the solver's own answer.
"""
import time

import numpy as np
import pytest

from paper_2307_01571_amd import qw
from paper_2307_01571_amd import surrogate as S
from paper_2307_01571_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


def test_generated_samples_are_the_solver_answers():
    print("[case] surrogate_generate runs=3 n=256 steps=300", flush=True)
    x, y, rid = S.generate(3, seed=7, steps=300, snap_every=100, n=256)
    wls = W.batch_instances(seed=7, count=3, sizes=(256,), steps=300)
    assert x.shape == (9, 5) and y.shape == (9, 6)
    for i, w in enumerate(wls):
        sim = qw.Sim(w.grid, qw.QW_F32, beam=w.beam)
        sim.init_packet(w.packet)
        for s in range(3):
            sim.step(100, s * 100 * W.DT, W.DT)
            ref = S.select_outputs(np.array(sim.observables(w.obs)))
            k = np.nonzero((rid == i))[0][s]
            assert np.allclose(x[k], [w.beam.w0, w.beam.a0, (s + 1) * 100 * W.DT, w.packet.p0y, w.packet.spin])
            assert np.max(np.abs(y[k] - ref)) <= 1e-12
        sim.close()


@pytest.mark.timeout(600)
def test_trained_surrogate_with_fallback():
    print("[case] surrogate_train runs=64 n=512 steps=2000", flush=True)
    x, y, rid = S.generate(64, seed=3, steps=2000, snap_every=200, n=512)
    held = rid >= 56
    net, hist = S.train(x[~held], y[~held], epochs=300, batch=256, lr=2e-3)
    assert hist[-1] < 0.5 * hist[0]  # standardised units: 1 = the constant predictor
    ev = S.evaluate(net, x[held], y[held])
    print("  held-out:", ev)
    assert ev["max_abs_all"] < 0.2
    # better than the constant predictor on the leading outputs
    assert ev["skill_vs_constant"][0] > 0.5 and ev["skill_vs_constant"][1] > 0.5
    pol = S.SurrogateWithFallback(net, tol=1e-2)
    # queries inside and far outside the training ranges (A0 = 3 was never seen)
    q = np.concatenate([x[held][:6], x[held][:2] * np.array([1, 0, 1, 1, 1]) + np.array([0, 3.0, 0, 0, 0])])
    out, used, spread = pol(q)
    ref = S.solve(q)
    assert np.all(np.abs(out[used] - ref[used]) == 0)
    print("  fallback used:", used, "spread:", spread)
    lat = S.latency(net, x[held][:4], reps=5)
    print("  latency:", lat)
    assert lat["speedup_1_query"] > 100
    net.close()
