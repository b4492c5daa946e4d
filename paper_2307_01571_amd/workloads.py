"""Seeded synthetic workloads shaped like the paper's simulations.

This module only states parameters (grid, field, packet, time step, step
count) and draws the seeded random ones.  It holds none of the method's
arithmetic, imports neither the HIP binding nor the oracle, and is the one
piece both the tests' oracle runs and the GPU runs take their inputs from.

Units are atomic units (m = hbar = |q| = 1, c = 137.036).  The paper's
showcase (Sec. II.D) uses a 2048 x 128 grid with a co-moving box; the
workloads here are square periodic boxes with the paraxial standing wave,
keeping the paper's structure: a Gaussian packet in momentum space (Eq. 12),
Bragg incidence p_x = -k_L (Sec. II.D) and diffraction into p_x + 2 n k_L.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict, replace
from typing import List

import numpy as np

C_AU = 137.036          # speed of light in atomic units
LAMBDA_L = 0.5          # laser wavelength (a.u.)
K_L = 2.0 * math.pi / LAMBDA_L
T_L = LAMBDA_L / C_AU   # laser period
DT = T_L / 64.0         # time step used by every workload
RAMP_PERIODS = 20.0     # sin^2 switch-on over 20 laser periods

PREC_F64 = 0
PREC_F32 = 1

BEAM_NONE = 0
BEAM_STANDING_PARAXIAL = 1
BEAM_UNIFORM = 2


@dataclass
class GridSpec:
    nx: int
    ny: int
    x_min: float
    y_min: float
    lx: float
    ly: float
    c: float = C_AU


@dataclass
class BeamSpec:
    mode: int = BEAM_STANDING_PARAXIAL
    a0: float = 0.5
    lambda_l: float = LAMBDA_L
    w0: float = 4 * LAMBDA_L
    ramp_periods: float = RAMP_PERIODS
    longitudinal: int = 1
    ux: float = 0.0
    uy: float = 0.0


@dataclass
class PacketSpec:
    p0x: float = -K_L
    p0y: float = 0.1 * K_L
    x0: float = 0.0
    y0: float = 0.0
    sigma_x: float = 3 * LAMBDA_L
    spin: int = 1


@dataclass
class ObsSpec:
    band_ref_idx: int      # p_ref / dk
    band_half_idx: int     # k_L / dk
    window_idx: int        # half-width of each diffraction window, in dk
    n_max: int = 2
    spin0: int = 1


@dataclass
class Workload:
    name: str
    grid: GridSpec
    beam: BeamSpec
    packet: PacketSpec
    obs: ObsSpec
    dt: float = DT
    steps: int = 200
    t0: float = 0.0
    meta: dict = field(default_factory=dict)

    def to_dict(self):
        return asdict(self)

    def with_steps(self, steps: int) -> "Workload":
        return replace(self, steps=int(steps))


def square_box(n: int, periods: int) -> GridSpec:
    """Square periodic box of `periods` laser wavelengths centred on the focus."""
    length = periods * LAMBDA_L
    return GridSpec(nx=n, ny=n, x_min=-0.5 * length, y_min=-0.5 * length, lx=length, ly=length)


def obs_for(grid: GridSpec, packet: PacketSpec, spin0: int = 1, n_max: int = 2) -> ObsSpec:
    """Diffraction windows of half-width k_L / 2 about p_ref + 2 n k_L, p_ref = p0x.

    Everything is in units of the grid's dk = 2 pi / lx; k_L / dk = lx / lambda_L
    must be an integer so the window centres fall on grid lines.
    """
    m = grid.lx / LAMBDA_L
    if abs(m - round(m)) > 1e-9:
        raise ValueError("box length must be a whole number of wavelengths")
    m = int(round(m))
    r = packet.p0x / (2.0 * math.pi / grid.lx)
    return ObsSpec(band_ref_idx=int(round(r)), band_half_idx=m, window_idx=m // 2, n_max=n_max, spin0=spin0)


def small_parity() -> Workload:
    """64 x 64, box 16 lambda, w0 = 4 lambda, A0 = 0.5, 200 steps (FP64 parity case)."""
    g = square_box(64, 16)
    b = BeamSpec(a0=0.5, w0=4 * LAMBDA_L)
    p = PacketSpec()
    return Workload("grid64_box16_w4_a0.5_200steps", g, b, p, obs_for(g, p), steps=200)


def mid_instances(seed: int = 0) -> List[Workload]:
    """512 x 512, box 16 lambda, w0 in {2, 4, 8} lambda, A0 ~ U[0.1, 1.0] (seeded), 1e4 steps."""
    rng = np.random.default_rng(seed)
    out = []
    for w in (2, 4, 8):
        a0 = float(rng.uniform(0.1, 1.0))
        g = square_box(512, 16)
        b = BeamSpec(a0=a0, w0=w * LAMBDA_L)
        p = PacketSpec()
        out.append(Workload(f"grid512_box16_w{w}_a0{a0:.4f}_1e4steps", g, b, p, obs_for(g, p),
                            steps=10_000, meta={"seed": seed, "a0_draw": a0}))
    return out


def large() -> Workload:
    """2048 x 2048, box 64 lambda, w0 = 16 lambda, A0 = 0.5, 5e4 steps (throughput case)."""
    g = square_box(2048, 64)
    b = BeamSpec(a0=0.5, w0=16 * LAMBDA_L)
    p = PacketSpec()
    return Workload("grid2048_box64_w16_a0.5_5e4steps", g, b, p, obs_for(g, p), steps=50_000)


def batch_instances(seed: int = 0, count: int = 96, sizes=(256, 512, 1024), steps: int = 20_000,
                    p0y_max: float = 0.3) -> List[Workload]:
    """Batching workload: `count` independent instances with seeded parameters.

    Per instance, in this draw order: N uniform over `sizes` (square N x N
    grid with dx = lambda/32, so the box is N/32 wavelengths), w0 ~ U[2, 16]
    lambda, A0 ~ U[0.05, 1.0], p0y ~ U[0, p0y_max] k_L, spin +1 or -1 with
    probability 1/2.  Packet at p0x = -k_L, sigma_x = 3 lambda, centred on
    the focus; dt = T_L/64; `steps` steps each.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(sizes[int(rng.integers(len(sizes)))])
        w0 = float(rng.uniform(2.0, 16.0)) * LAMBDA_L
        a0 = float(rng.uniform(0.05, 1.0))
        p0y = float(rng.uniform(0.0, p0y_max)) * K_L
        spin = 1 if rng.random() < 0.5 else -1
        g = square_box(n, n // 32)
        b = BeamSpec(a0=a0, w0=w0)
        p = PacketSpec(p0y=p0y, spin=spin)
        out.append(Workload(f"batch{i}_grid{n}_w{w0 / LAMBDA_L:.3f}_a{a0:.4f}_py{p0y / K_L:.4f}_s{spin:+d}",
                            g, b, p, obs_for(g, p, spin0=spin), steps=steps,
                            meta={"seed": seed, "index": i}))
    return out


# ---- learned form: the surrogate network's shape, input map and seeded start ----
SURROGATE_SHAPE = dict(n_in=5, width=256, depth=4, n_out=6, n_nets=4)
# inputs (w0, A0, interaction time, p0y, spin) are mapped to about [-1, 1]
# by (x - shift) * scale over the ranges the batching workload draws from
SURROGATE_INPUT_RANGES = ((2.0 * LAMBDA_L, 16.0 * LAMBDA_L), (0.05, 1.0), (0.0, 20_000 * DT),
                          (0.0, 0.3 * K_L), (-1.0, 1.0))
SURROGATE_OUTPUTS = ("P_0", "P_+1", "P_-1", "P_+2", "P_-2", "P_flip")


def surrogate_input_map():
    """(shift, scale) of the surrogate's input normalisation."""
    shift = np.array([(lo + hi) / 2 for lo, hi in SURROGATE_INPUT_RANGES])
    scale = np.array([2.0 / (hi - lo) for lo, hi in SURROGATE_INPUT_RANGES])
    return shift, scale


def mlp_layer_sizes(n_in: int, width: int, depth: int, n_out: int):
    """(out, in) of every linear layer of an MLP with `depth` hidden layers."""
    return [(width, n_in)] + [(width, width)] * (depth - 1) + [(n_out, width)]


def mlp_init_params(seed: int, n_in: int, width: int, depth: int, n_out: int) -> np.ndarray:
    """Seeded initial parameters, flat: per layer W[out][in] row-major then b[out];
    W ~ U(-1/sqrt(in), 1/sqrt(in)), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for no, ni in mlp_layer_sizes(n_in, width, depth, n_out):
        lim = 1.0 / math.sqrt(ni)
        parts.append(rng.uniform(-lim, lim, size=no * ni))
        parts.append(np.zeros(no))
    return np.concatenate(parts)


def random_state(ny: int, nx: int, seed: int, ncomp: int = 4) -> np.ndarray:
    """Seeded complex128 test state with unit norm (not a physical packet)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((ny, nx, ncomp)) + 1j * rng.standard_normal((ny, nx, ncomp))
    return a / np.sqrt(np.sum(np.abs(a) ** 2))
