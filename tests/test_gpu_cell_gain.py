"""Norm gain of single momentum cells under the FP32 free step, against the
exact model of the float transform pair (host arithmetic in
tests/test_transform_gain.py), through the C ABI.

A plane wave exp(2 pi i k x / nx) in one spinor component stays in its
momentum cell under the free step (field off); its norm changes only by the
step's rounding.  Most of that change is the same for every cell or the same
for +-k (the kinetic step is symmetric in +-kx), but the round trip of the x
transforms with float-rounded constants gives each cell its own gain, and
cells +k and -k differ by what the model of that round trip gives: for 2048
points 1.21e-7 per step at k = 1 and 5.8e-8 at k = 80 with the plain constants,
a few 1e-9 with split (hi + lo) rotation constants.  The measured difference
of the kernels must match the model of the constant set the library was
built with.  FP64 gains stay at rounding level.
"""
import math

import numpy as np
import pytest

from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W
from test_transform_gain import PLANS_F32, split_build, stockham

pytestmark = pytest.mark.gpu

NX, NY, STEPS = 2048, 16, 20_000


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (HIP device)")
    qw.lib()


@pytest.fixture(scope="module")
def model_gain():
    """|g(k)|^2 of the x round trip (inverse then forward, 1/N) for all k."""
    F = stockham(np.eye(NX, dtype=complex), PLANS_F32[NX], f32=True, split_rotations=split_build())
    Fi = np.conj(F)
    g = np.einsum("kj,jk->k", F, Fi) / NX
    return np.abs(g) ** 2


def cell_gain(prec, kx, comp=0):
    import torch
    g = W.GridSpec(nx=NX, ny=NY, x_min=-40 * W.LAMBDA_L, y_min=-5 * W.LAMBDA_L, lx=80 * W.LAMBDA_L,
                   ly=10 * W.LAMBDA_L)
    sim = qw.Sim(g, prec, beam=W.BeamSpec(mode=qw.QW_BEAM_NONE))
    ix = torch.arange(NX, dtype=torch.float64, device="cuda")
    w = torch.zeros((NY, NX, 4), dtype=torch.complex128, device="cuda")
    w[:, :, comp] = torch.exp(2j * math.pi * kx * ix / NX)[None, :] / math.sqrt(NX * NY)
    sim.psi.copy_(w.to(sim.psi.dtype))
    n0 = float((sim.psi.to(torch.complex128).abs() ** 2).sum())
    sim.step(STEPS, 0.0, W.DT)
    torch.cuda.synchronize()
    n1 = float((sim.psi.to(torch.complex128).abs() ** 2).sum())
    sim.close()
    return math.log(n1 / n0) / STEPS


@pytest.mark.parametrize("k", [1, 80])
def test_cell_gain_difference_matches_the_transform_model(k, model_gain):
    print(f"[case] cell gain +-{k}, {NX}x{NY} FP32, {STEPS} free steps", flush=True)
    plus = [cell_gain(qw.QW_F32, k, c) for c in (0, 3)]
    minus = [cell_gain(qw.QW_F32, -k, c) for c in (0, 3)]
    meas = np.mean(plus) - np.mean(minus)
    model = model_gain[k] - model_gain[-k]
    print(f"  gain +{k}: {plus}, -{k}: {minus}; difference {meas:+.3e}, model {model:+.3e}")
    # the same for every component, to a few 1e-9 of rounding noise over these steps
    assert abs(plus[0] - plus[1]) < 1e-8 and abs(minus[0] - minus[1]) < 1e-8
    if split_build():
        assert abs(meas) < 1.5e-8
    else:
        assert abs(model) > 5e-8
        assert abs(meas - model) < 0.1 * abs(model)


def test_cell_gain_in_double_is_rounding_level():
    print(f"[case] cell gain FP64, {NX}x{NY}, {STEPS} free steps", flush=True)
    for k in (1, -80):
        assert abs(cell_gain(qw.QW_F64, k)) < 1e-14
