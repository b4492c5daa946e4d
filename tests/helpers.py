"""Test helpers: convert the seeded workload specs into oracle inputs."""
import numpy as np

import oracle
from paper_2307_01571_amd import workloads as W


def o_grid(g: W.GridSpec) -> oracle.Grid:
    return oracle.Grid(g.nx, g.ny, g.x_min, g.y_min, g.lx, g.ly, g.c)


def o_beam(b: W.BeamSpec) -> oracle.Beam:
    return oracle.Beam(b.mode, b.a0, b.lambda_l, b.w0, b.ramp_periods, b.longitudinal, b.ux, b.uy)


def o_packet(p: W.PacketSpec) -> oracle.Packet:
    return oracle.Packet(p.p0x, p.p0y, p.x0, p.y0, p.sigma_x, p.spin)


def o_obs(o: W.ObsSpec) -> oracle.ObsSpec:
    return oracle.ObsSpec(o.band_ref_idx, o.band_half_idx, o.window_idx, o.n_max, o.spin0)


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def momenta(g: W.GridSpec):
    """Momentum grid of the FFT ordering (numpy's fftfreq puts the Nyquist mode at -n/2)."""
    px = 2 * np.pi * np.fft.fftfreq(g.nx, d=g.lx / g.nx)
    py = 2 * np.pi * np.fft.fftfreq(g.ny, d=g.ly / g.ny)
    return np.meshgrid(px, py)  # arrays of shape (ny, nx)
