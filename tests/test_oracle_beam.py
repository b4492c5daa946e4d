"""Pins of the oracle's vector potential.

The paper's field (Sec. II.A, Eq. 1-4) is the superposition of two
counter-propagating Gaussian beams with Gouy and curvature phases.  The
oracle evaluates its paraxial (x << x_R) standing-wave form.  The pins:
  * it equals the paper's full Eq. 1-4, written out independently below, as
    x / x_R -> 0, with amplitude A0 = 2 A0_paper and the paper's time shifted
    by a quarter period (the paper has sin(w t), the standing wave here cos(w t));
  * the field is divergence free (Coulomb gauge, as the paper states);
  * the sin^2 switch-on makes A vanish at t = 0 and reach full strength after
    the ramp.
"""
import math

import numpy as np
import pytest

import oracle

C = 137.036
LAM = 0.5
KL = 2 * math.pi / LAM
OM = C * KL
TL = LAM / C


def paper_beam(x, y, t, a0_paper, eps, longitudinal=True):
    """Eq. 1a, 1b, 2, 3, 4 of the paper at z = 0 (r^2 = y^2), summed over d = +-1."""
    w0 = 1.0 / (KL * eps)
    xr = KL * w0 * w0 / 2.0
    w = w0 * math.sqrt(1 + x * x / (xr * xr))
    ax = ay = 0.0
    for d in (-1, 1):
        phi = OM * t - d * KL * x + math.atan(d * x / xr) - d * x * y * y / (xr * w * w)
        phi1 = phi + math.atan(d * x / xr)
        env = (w0 / w) * math.exp(-y * y / (w * w))
        ay += -a0_paper * env * math.sin(phi)
        if longitudinal:
            ax += -2 * d * a0_paper * env * eps * (y / w) * math.cos(phi1)
    return ax, ay


@pytest.mark.parametrize("longitudinal", [1, 0])
def test_paraxial_limit_of_paper_beam(longitudinal):
    eps = 2e-3
    w0 = 1.0 / (KL * eps)
    xr = KL * w0 * w0 / 2
    a0 = 0.5
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=a0, lambda_l=LAM, w0=w0,
                       ramp_periods=0.0, longitudinal=longitudinal)
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(200):
        x = rng.uniform(-4 * LAM, 4 * LAM)
        y = rng.uniform(-1.5 * w0, 1.5 * w0)
        t = rng.uniform(0, 5 * TL)
        ax, ay = oracle.beam_eval(beam, C, x, y, t)
        px, py = paper_beam(x, y, t - TL / 4, a0 / 2, eps, bool(longitudinal))
        # each component against its own scale: A_y ~ A0, A_x ~ A0 eps
        worst = max(worst, abs(ax - px) / (a0 * eps), abs(ay - py) / a0)
    # deviation is O(x / x_R) (Gouy and curvature phases, w(x) - w0)
    assert worst <= 4 * (4 * LAM) / xr
    assert 4 * LAM / xr < 1e-3


def test_sign_flip_is_caught_by_paraxial_pin():
    """The pin above is sharp: the paper beam with the opposite sign disagrees at O(1)."""
    eps = 2e-3
    w0 = 1.0 / (KL * eps)
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=0.5, lambda_l=LAM, w0=w0, ramp_periods=0.0)
    x, y, t = 0.3, 0.4 * w0, 0.37 * TL
    ax, ay = oracle.beam_eval(beam, C, x, y, t)
    px, py = paper_beam(x, y, t - TL / 4, 0.25, eps)
    assert abs(ay - py) < 1e-3 * 0.5 and abs(ax - px) < 1e-3 * 0.5 * eps
    assert abs(ay + py) > 0.1 * 0.5 and abs(ax + px) > 0.1 * 0.5 * eps


def test_divergence_free():
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=0.8, lambda_l=LAM, w0=2 * LAM,
                       ramp_periods=20.0, longitudinal=1)
    rng = np.random.default_rng(5)
    h = 1e-4
    for _ in range(50):
        x, y = rng.uniform(-3, 3, size=2)
        t = rng.uniform(0, 40 * TL)

        def f(xx, yy):
            return oracle.beam_eval(beam, C, xx, yy, t)
        # fourth-order central differences
        dax = (-f(x + 2 * h, y)[0] + 8 * f(x + h, y)[0] - 8 * f(x - h, y)[0] + f(x - 2 * h, y)[0]) / (12 * h)
        day = (-f(x, y + 2 * h)[1] + 8 * f(x, y + h)[1] - 8 * f(x, y - h)[1] + f(x, y - 2 * h)[1]) / (12 * h)
        scale = 0.8 * KL
        assert abs(dax + day) <= 1e-8 * scale
    # and the longitudinal part is needed for that: without it the divergence is O(A0 / w0)
    b2 = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=0.8, lambda_l=LAM, w0=2 * LAM,
                     ramp_periods=0.0, longitudinal=0)
    x, y, t = 0.1, 0.7, 0.0
    day = (oracle.beam_eval(b2, C, x, y + h, t)[1] - oracle.beam_eval(b2, C, x, y - h, t)[1]) / (2 * h)
    assert abs(day) > 0.1


def test_ramp():
    beam = oracle.Beam(mode=oracle.BEAM_STANDING_PARAXIAL, a0=0.5, lambda_l=LAM, w0=2.0,
                       ramp_periods=20.0, longitudinal=1)
    assert oracle.beam_eval(beam, C, 0.0, 0.3, 0.0) == (0.0, 0.0)
    tr = 20 * TL
    # after the ramp the amplitude at x = y = 0 is A0 cos(w t)
    for t in (tr, tr + 0.3 * TL, 3 * tr):
        ax, ay = oracle.beam_eval(beam, C, 0.0, 0.0, t)
        assert abs(ay - 0.5 * math.cos(OM * t)) <= 1e-14 and ax == 0.0
    # half-way through the ramp: sin^2(pi/4) = 1/2, at a crest of cos(w t) (t = 10 T_L)
    ax, ay = oracle.beam_eval(beam, C, 0.0, 0.0, 10 * TL)
    assert abs(ay - 0.25) <= 1e-12


def test_uniform_and_none_modes():
    b = oracle.Beam(mode=oracle.BEAM_UNIFORM, ux=0.3, uy=-0.2)
    assert oracle.beam_eval(b, C, 1.0, 2.0, 3.0) == (0.3, -0.2)
    b = oracle.Beam(mode=oracle.BEAM_NONE, a0=1.0)
    assert oracle.beam_eval(b, C, 1.0, 2.0, 3.0) == (0.0, 0.0)
