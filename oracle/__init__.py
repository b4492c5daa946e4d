"""The oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU implementation of the Dirac FFT split-operator method
(Ge, Ahrens, Shen, Sec. II, Eq. 1-15; observables Sec. III.B, Eq. 18-19),
written in C (``qw_oracle.c``) and wrapped here with ctypes for numpy arrays.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it and
shares no code with it.  Every function here is a thin marshalling layer;
all arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "qw_oracle.c")

BEAM_NONE = 0
BEAM_STANDING_PARAXIAL = 1
BEAM_UNIFORM = 2
BEAM_GAUSSIAN_FULL = 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math), OpenMP on."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x_min", ctypes.c_double), ("y_min", ctypes.c_double),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("c", ctypes.c_double)]


class _Beam(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("a0", ctypes.c_double),
                ("lambda_l", ctypes.c_double), ("w0", ctypes.c_double),
                ("ramp_periods", ctypes.c_double), ("longitudinal", ctypes.c_int),
                ("ux", ctypes.c_double), ("uy", ctypes.c_double)]


class _Packet(ctypes.Structure):
    _fields_ = [("p0x", ctypes.c_double), ("p0y", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("sigma_x", ctypes.c_double), ("spin", ctypes.c_int)]


class _Frame(ctypes.Structure):
    _fields_ = [("vy", ctypes.c_double), ("a_m", ctypes.c_double)]


class _Obs(ctypes.Structure):
    _fields_ = [("band_ref_idx", ctypes.c_int), ("band_half_idx", ctypes.c_int),
                ("window_idx", ctypes.c_int), ("n_max", ctypes.c_int), ("spin0", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_fft1d.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        L.or_dft2.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_beam_eval.argtypes = [ctypes.POINTER(_Beam), ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_beam_eval.restype = None
        L.or_step_n.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Beam), dp,
                                ctypes.c_long, ctypes.c_double, ctypes.c_double]
        L.or_spinor.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        L.or_spinor.restype = None
        L.or_init_packet.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Packet), dp]
        L.or_step_n_frame.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Beam), ctypes.POINTER(_Frame), dp,
                                      ctypes.c_long, ctypes.c_double, ctypes.c_double]
        L.or_init_packet_frame.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Packet), ctypes.POINTER(_Frame),
                                           dp]
        L.or_observables_frame.argtypes = [ctypes.POINTER(_Grid), dp, ctypes.POINTER(_Obs), ctypes.POINTER(_Frame),
                                           dp, ctypes.c_int]
        L.or_band_index.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_observables.argtypes = [ctypes.POINTER(_Grid), dp, ctypes.POINTER(_Obs), dp, ctypes.c_int]
        for name in ("or_hamiltonian0", "or_kinetic_matrix"):
            getattr(L, name).restype = None
        L.or_hamiltonian0.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.or_kinetic_matrix.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, dp]
        L.or_interaction_matrix.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, dp]
        L.or_interaction_matrix.restype = None
        L.or_energy.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_energy.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    nx: int
    ny: int
    x_min: float
    y_min: float
    lx: float
    ly: float
    c: float

    def cstruct(self):
        return _Grid(self.nx, self.ny, self.x_min, self.y_min, self.lx, self.ly, self.c)


@dataclass
class Beam:
    mode: int = BEAM_STANDING_PARAXIAL
    a0: float = 0.0
    lambda_l: float = 0.5
    w0: float = 2.0
    ramp_periods: float = 20.0
    longitudinal: int = 1
    ux: float = 0.0
    uy: float = 0.0

    def cstruct(self):
        return _Beam(self.mode, self.a0, self.lambda_l, self.w0, self.ramp_periods,
                     self.longitudinal, self.ux, self.uy)


@dataclass
class Packet:
    p0x: float
    p0y: float
    x0: float
    y0: float
    sigma_x: float
    spin: int = 1

    def cstruct(self):
        return _Packet(self.p0x, self.p0y, self.x0, self.y0, self.sigma_x, self.spin)


@dataclass
class Frame:
    """Box moving along y with velocity vy, constant gauge vector potential a_m along y."""
    vy: float = 0.0
    a_m: float = 0.0

    def cstruct(self):
        return _Frame(self.vy, self.a_m)


@dataclass
class ObsSpec:
    band_ref_idx: int
    band_half_idx: int
    window_idx: int
    n_max: int = 2
    spin0: int = 1

    def cstruct(self):
        return _Obs(self.band_ref_idx, self.band_half_idx, self.window_idx, self.n_max, self.spin0)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def fft1d(x: np.ndarray, sign: int = -1) -> np.ndarray:
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    _check(lib().or_fft1d(_ptr(a), a.shape[0], sign), "fft1d")
    return a


def dft2(psi: np.ndarray, sign: int = -1) -> np.ndarray:
    """2D transform of a (ny, nx, ncomp) array; sign=+1 includes 1/(nx ny)."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    if a.ndim == 2:
        a = a[:, :, None].copy()
    ny, nx, nc = a.shape
    _check(lib().or_dft2(_ptr(a), nx, ny, nc, sign), "dft2")
    return a.reshape(psi.shape)


def beam_eval(beam: Beam, c: float, x: float, y: float, t: float):
    ax = ctypes.c_double()
    ay = ctypes.c_double()
    b = beam.cstruct()
    lib().or_beam_eval(ctypes.byref(b), c, x, y, t, ctypes.byref(ax), ctypes.byref(ay))
    return ax.value, ay.value


def init_packet(grid: Grid, packet: Packet, frame: Frame = None) -> np.ndarray:
    psi = np.zeros((grid.ny, grid.nx, 4), dtype=np.complex128)
    g = grid.cstruct()
    e = packet.cstruct()
    if frame is None:
        _check(lib().or_init_packet(ctypes.byref(g), ctypes.byref(e), _ptr(psi)), "init_packet")
    else:
        f = frame.cstruct()
        _check(lib().or_init_packet_frame(ctypes.byref(g), ctypes.byref(e), ctypes.byref(f), _ptr(psi)),
               "init_packet")
    return psi


def step_n(grid: Grid, beam: Beam, psi: np.ndarray, n: int, t0: float, dt: float, frame: Frame = None) -> np.ndarray:
    """Return psi after n split-operator steps from t0 (the input is not modified)."""
    a = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    assert a.shape == (grid.ny, grid.nx, 4)
    g = grid.cstruct()
    b = beam.cstruct()
    if frame is None:
        rc = lib().or_step_n(ctypes.byref(g), ctypes.byref(b), _ptr(a), int(n), float(t0), float(dt))
    else:
        f = frame.cstruct()
        rc = lib().or_step_n_frame(ctypes.byref(g), ctypes.byref(b), ctypes.byref(f), _ptr(a), int(n), float(t0),
                                   float(dt))
    _check(rc, "step_n")
    return a


def observables(grid: Grid, psi: np.ndarray, spec: ObsSpec, frame: Frame = None) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    nb = 2 * spec.n_max + 1
    out = np.zeros(3 * nb + 3, dtype=np.float64)
    g = grid.cstruct()
    o = spec.cstruct()
    if frame is None:
        rc = lib().or_observables(ctypes.byref(g), _ptr(a), ctypes.byref(o), _ptr(out), out.size)
    else:
        f = frame.cstruct()
        rc = lib().or_observables_frame(ctypes.byref(g), _ptr(a), ctypes.byref(o), ctypes.byref(f), _ptr(out),
                                        out.size)
    if rc not in (0, -5):
        raise RuntimeError(f"oracle observables failed with status {rc}")
    return out


def spinor(px: float, py: float, c: float, s: int) -> np.ndarray:
    u = np.zeros(4, dtype=np.complex128)
    lib().or_spinor(px, py, c, s, _ptr(u))
    return u


NO_BAND = -(1 << 30)


def band_index(kx_signed: int, ref_idx: int, half_idx: int, window_idx: int) -> int:
    """Diffraction order of a momentum column, or NO_BAND outside every window."""
    return int(lib().or_band_index(kx_signed, ref_idx, half_idx, window_idx))


def _mat(fn, *args) -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    fn(*args, _ptr(m))
    return m


def hamiltonian0(px: float, py: float, c: float) -> np.ndarray:
    return _mat(lib().or_hamiltonian0, px, py, c)


def kinetic_matrix(px: float, py: float, c: float, tau: float) -> np.ndarray:
    return _mat(lib().or_kinetic_matrix, px, py, c, tau)


def interaction_matrix(ax: float, ay: float, c: float, tau: float) -> np.ndarray:
    return _mat(lib().or_interaction_matrix, ax, ay, c, tau)


def energy(px: float, py: float, c: float) -> float:
    return float(lib().or_energy(px, py, c))


def unpack_observables(out: np.ndarray, n_max: int) -> dict:
    nb = 2 * n_max + 1
    return {
        "norm": float(out[0]),
        "P": out[1:1 + nb].copy(),
        "Pp": out[1 + nb:1 + 2 * nb].copy(),
        "Pm": out[1 + 2 * nb:1 + 3 * nb].copy(),
        "P_flip": float(out[1 + 3 * nb]),
        "P_neg": float(out[2 + 3 * nb]),
    }
