"""Host-side checks of the paper-fidelity set-ups (Sec. II.D): the showcase
parameters in atomic units and the derived step count, box and packet."""
import math

from paper_2307_01571_amd import experiments as X
from paper_2307_01571_amd import qw
from paper_2307_01571_amd import workloads as W

C = W.C_AU


def test_showcase_parameters():
    cfg = X.setup()
    g, b, p = cfg["grid"], cfg["beam"], cfg["packet"]
    lam = 2 * math.pi / (0.1 * C)
    assert (g.nx, g.ny) == (2048, 128)
    assert abs(g.lx - 80 * lam) < 1e-12 and abs(g.ly - 40 * lam) < 1e-12
    assert abs(g.x_min + 40 * lam) < 1e-12 and abs(g.y_min + 160 * lam) < 1e-12
    assert b.mode == qw.QW_BEAM_GAUSSIAN_FULL and abs(b.a0 - 0.1 * C) < 1e-12
    assert abs(1 / (b.w0 * 0.1 * C) - 0.02) < 1e-15                      # eps
    assert abs(p.p0x + 0.1 * C) < 1e-12 and abs(p.p0y - C) < 1e-12          # (-hbar k_L, m c)
    assert abs(p.x0 - 140 * 2 * math.pi / C) < 1e-12 and abs(p.y0 + 140 * lam) < 1e-12
    assert abs(1 / (2 * p.sigma_x) - 0.1 * C / 200) < 1e-12                 # sigma_p = hbar k_L / 200
    assert abs(cfg["dt"] - 0.05 / C ** 2) < 1e-20
    # travel time 280 lambda sqrt2 / c = 2.5e4 hbar/(m c^2): about 5e5 steps
    assert abs(cfg["steps"] * cfg["dt"] * C ** 2 - 280 * lam * math.sqrt(2) * C) < 0.05
    assert 4.9e5 < cfg["steps"] < 5.1e5
    assert abs(cfg["vy"] - C / math.sqrt(2)) < 1e-12 and cfg["a_m"] == C
    o = cfg["obs"]
    assert o.band_half_idx == 80 and o.band_ref_idx == -80


def test_scan_step_counts_scale_with_the_wavelength():
    n = {kl: X.setup(kl_mc=kl)["steps"] for kl in (0.05, 0.07, 0.1)}
    assert abs(n[0.05] / n[0.1] - 2.0) < 1e-4
    assert abs(n[0.07] / n[0.1] - 0.1 / 0.07) < 1e-4


def test_diffraction_setup():
    cfg = X.setup(kl_mc=0.1, eps=0.1, a0_mc=0.4, ny=256, px_kl=0.0)
    assert cfg["grid"].ny == 256 and abs(cfg["beam"].a0 - 0.4 * C) < 1e-12
    assert cfg["packet"].p0x == 0.0 and cfg["obs"].band_ref_idx == 0


def test_loglog_slope():
    assert abs(X.loglog_slope([1, 2, 4], [3, 12, 48]) - 2.0) < 1e-12
