"""ctypes binding of libqw.so (include/qw.h) -- argument marshalling only.

The functions below carry the C names and forward to the library; every
step of the computation runs in the library's HIP kernels.  There is no
fallback: if libqw.so is missing or cannot be loaded, ``lib()`` raises.

``Sim`` is a convenience owner of the torch tensors (state and workspace) on
one device; torch is used only as the device allocator and for streams.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import asdict
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqw.so")

QW_OK = 0
QW_E_ARG = -1
QW_E_SIZE = -2
QW_E_WORKSPACE = -3
QW_E_DEVICE = -4
QW_E_NUMERIC = -5
QW_E_STATE = -6

QW_F64 = 0
QW_F32 = 1
QW_MLP_STATIC_MAX_BATCH = 256  # qw_mlp.h

QW_LOOP_INSTANCE = -2  # qw_batch_set_loop: one workgroup per instance

QW_BEAM_NONE = 0
QW_BEAM_STANDING_PARAXIAL = 1
QW_BEAM_UNIFORM = 2
QW_BEAM_GAUSSIAN_FULL = 3

EXPORTED = ("qw_workspace_bytes", "qw_init_grid", "qw_set_beam", "qw_set_frame", "qw_init_packet", "qw_step_n",
            "qw_observables", "qw_momentum_maps", "qw_kernel_timing", "qw_kernel_times", "qw_transform_gain", "qw_last_error",
            "qw_destroy",
            "qw_batch_layout", "qw_batch_init", "qw_batch_init_packets", "qw_batch_step_n",
            "qw_batch_observables", "qw_batch_schedule", "qw_batch_set_schedule", "qw_batch_set_launch",
            "qw_batch_set_loop", "qw_batch_autotune", "qw_batch_kernel_timing", "qw_batch_kernel_times", "qw_batch_last_error",
            "qw_batch_destroy",
            "qw_mlp_param_count", "qw_mlp_workspace_bytes", "qw_mlp_init", "qw_mlp_set_params",
            "qw_mlp_set_output_map", "qw_mlp_set_spread_weights", "qw_mlp_get_params", "qw_mlp_forward", "qw_mlp_predict", "qw_mlp_predict_static",
            "qw_mlp_gradients", "qw_mlp_train_step",
            "qw_gemm_bf16_nt", "qw_mlp_last_error", "qw_mlp_destroy")
_NO_STATUS = ("qw_last_error", "qw_destroy", "qw_batch_last_error", "qw_batch_destroy", "qw_mlp_last_error",
              "qw_mlp_destroy")


class qw_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("y_min", ctypes.c_double),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("c", ctypes.c_double), ("precision", ctypes.c_int32)]


class qw_beam(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("a0", ctypes.c_double), ("lambda_l", ctypes.c_double),
                ("w0", ctypes.c_double), ("ramp_periods", ctypes.c_double),
                ("longitudinal", ctypes.c_int32), ("ux", ctypes.c_double), ("uy", ctypes.c_double)]


class qw_frame(ctypes.Structure):
    _fields_ = [("vy", ctypes.c_double), ("a_m", ctypes.c_double)]


class qw_packet(ctypes.Structure):
    _fields_ = [("p0x", ctypes.c_double), ("p0y", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("sigma_x", ctypes.c_double), ("spin", ctypes.c_int32)]


class qw_obs_spec(ctypes.Structure):
    _fields_ = [("band_ref_idx", ctypes.c_int32), ("band_half_idx", ctypes.c_int32),
                ("window_idx", ctypes.c_int32), ("n_max", ctypes.c_int32), ("spin0", ctypes.c_int32)]


class qw_instance(ctypes.Structure):
    _fields_ = [("grid", qw_grid), ("beam", qw_beam)]


class qw_mlp_shape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("n_nets", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


_lib = None


def lib():
    """Load libqw.so (built by ``paper_2307_01571_amd.build``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_01571_amd.build`")
    # torch ships its own HIP runtime under another file name; loading torch
    # first makes the library bind to that same runtime (same SONAME) instead
    # of a second copy, so both see the same devices and allocations
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.qw_workspace_bytes.argtypes = [ctypes.POINTER(qw_grid), ctypes.POINTER(ctypes.c_size_t)]
    L.qw_init_grid.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(qw_grid), vp, ctypes.c_size_t, vp]
    L.qw_set_beam.argtypes = [vp, ctypes.POINTER(qw_beam)]
    L.qw_set_frame.argtypes = [vp, ctypes.POINTER(qw_frame)]
    L.qw_init_packet.argtypes = [vp, vp, ctypes.POINTER(qw_packet), vp]
    L.qw_step_n.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, vp]
    L.qw_observables.argtypes = [vp, vp, ctypes.POINTER(qw_obs_spec), dp, ctypes.c_int32, vp]
    L.qw_momentum_maps.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
    L.qw_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.qw_kernel_times.argtypes = [vp, dp, ctypes.c_int32, vp]
    L.qw_transform_gain.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp]
    L.qw_last_error.argtypes = [vp]
    L.qw_last_error.restype = ctypes.c_char_p
    L.qw_destroy.argtypes = [vp]
    L.qw_destroy.restype = None
    ip = ctypes.POINTER(qw_instance)
    i32p = ctypes.POINTER(ctypes.c_int32)
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.qw_batch_layout.argtypes = [ip, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), szp, szp]
    L.qw_batch_init.argtypes = [ctypes.POINTER(vp), ip, ctypes.c_int32, vp, ctypes.c_size_t, vp]
    L.qw_batch_init_packets.argtypes = [vp, vp, ctypes.POINTER(qw_packet), vp]
    L.qw_batch_step_n.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, vp]
    L.qw_batch_observables.argtypes = [vp, vp, ctypes.POINTER(qw_obs_spec), dp, ctypes.c_int32, vp]
    L.qw_batch_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, i32p, ctypes.c_int32]
    L.qw_batch_set_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.qw_batch_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.qw_batch_set_loop.argtypes = [vp, ctypes.c_int32, ctypes.c_double, i32p]
    L.qw_batch_autotune.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int32, dp, ctypes.c_int32, i32p, vp]
    L.qw_batch_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.qw_batch_kernel_times.argtypes = [vp, dp, ctypes.c_int32, vp]
    L.qw_batch_last_error.argtypes = [vp]
    L.qw_batch_last_error.restype = ctypes.c_char_p
    L.qw_batch_destroy.argtypes = [vp]
    L.qw_batch_destroy.restype = None
    shp = ctypes.POINTER(qw_mlp_shape)
    fp = ctypes.POINTER(ctypes.c_float)
    L.qw_mlp_param_count.argtypes = [shp, ctypes.POINTER(ctypes.c_int64)]
    L.qw_mlp_workspace_bytes.argtypes = [shp, szp]
    L.qw_mlp_init.argtypes = [ctypes.POINTER(vp), shp, fp, fp, vp, ctypes.c_size_t, vp]
    L.qw_mlp_set_params.argtypes = [vp, vp, vp]
    L.qw_mlp_get_params.argtypes = [vp, vp, vp]
    L.qw_mlp_set_output_map.argtypes = [vp, fp, fp, vp]
    L.qw_mlp_set_spread_weights.argtypes = [vp, fp, vp]
    L.qw_mlp_forward.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
    L.qw_mlp_predict.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.qw_mlp_predict_static.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.qw_mlp_gradients.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    L.qw_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp, vp]
    L.qw_gemm_bf16_nt.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, vp]
    L.qw_mlp_last_error.argtypes = [vp]
    L.qw_mlp_last_error.restype = ctypes.c_char_p
    L.qw_mlp_destroy.argtypes = [vp]
    L.qw_mlp_destroy.restype = None
    for name in EXPORTED:
        if name not in _NO_STATUS:
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class QWError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qw status {code}: {msg}")
        self.code = code


def _check(rc: int, ctx=None):
    if rc != QW_OK:
        raise QWError(rc, qw_last_error(ctx))


# ---- C names, marshalling only -------------------------------------------
def qw_workspace_bytes(grid: qw_grid) -> int:
    n = ctypes.c_size_t()
    _check(lib().qw_workspace_bytes(ctypes.byref(grid), ctypes.byref(n)))
    return n.value


def qw_init_grid(grid: qw_grid, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().qw_init_grid(ctypes.byref(h), ctypes.byref(grid), ctypes.c_void_p(workspace_ptr),
                              ws_bytes, ctypes.c_void_p(stream)))
    return h.value


def qw_set_beam(ctx: int, beam: qw_beam) -> None:
    _check(lib().qw_set_beam(ctypes.c_void_p(ctx), ctypes.byref(beam)), ctx)


def qw_set_frame(ctx: int, frame: qw_frame) -> None:
    _check(lib().qw_set_frame(ctypes.c_void_p(ctx), ctypes.byref(frame)), ctx)


def qw_init_packet(ctx: int, psi_ptr: int, packet: qw_packet, stream: int) -> None:
    _check(lib().qw_init_packet(ctypes.c_void_p(ctx), ctypes.c_void_p(psi_ptr), ctypes.byref(packet),
                                ctypes.c_void_p(stream)), ctx)


def qw_step_n(ctx: int, psi_ptr: int, n: int, t0: float, dt: float, stream: int) -> None:
    _check(lib().qw_step_n(ctypes.c_void_p(ctx), ctypes.c_void_p(psi_ptr), int(n), float(t0), float(dt),
                           ctypes.c_void_p(stream)), ctx)


def qw_observables(ctx: int, psi_ptr: int, spec: qw_obs_spec, stream: int, check: bool = True):
    nb = 2 * spec.n_max + 1
    out = (ctypes.c_double * (3 * nb + 3))()
    rc = lib().qw_observables(ctypes.c_void_p(ctx), ctypes.c_void_p(psi_ptr), ctypes.byref(spec), out,
                              3 * nb + 3, ctypes.c_void_p(stream))
    if check:
        _check(rc, ctx)
    return rc, [float(v) for v in out]


def qw_momentum_maps(ctx: int, psi_ptr: int, out_ptr: int, out_len: int, stream: int) -> None:
    _check(lib().qw_momentum_maps(ctypes.c_void_p(ctx), ctypes.c_void_p(psi_ptr), ctypes.c_void_p(out_ptr),
                                  int(out_len), ctypes.c_void_p(stream)), ctx)


def qw_kernel_timing(ctx: int, enable: bool) -> None:
    _check(lib().qw_kernel_timing(ctypes.c_void_p(ctx), int(bool(enable))), ctx)


def qw_kernel_times(ctx: int, stream: int):
    out = (ctypes.c_double * 4)()
    _check(lib().qw_kernel_times(ctypes.c_void_p(ctx), out, 4, ctypes.c_void_p(stream)), ctx)
    return [float(v) for v in out]


def qw_transform_gain(n: int, precision: int, batch_variant: int = -1) -> float:
    """Modelled mean squared-norm gain of one transform of length n (host arithmetic only)."""
    out = ctypes.c_double()
    _check(lib().qw_transform_gain(int(n), int(precision), int(batch_variant), ctypes.byref(out)), None)
    return out.value


def qw_last_error(ctx=None) -> str:
    s = lib().qw_last_error(ctypes.c_void_p(ctx) if ctx else None)
    return s.decode() if s else ""


def qw_destroy(ctx: int) -> None:
    lib().qw_destroy(ctypes.c_void_p(ctx))


# ---- batched form -----------------------------------------------------------
class QWBatchError(QWError):
    pass


def _bcheck(rc: int, b=None):
    if rc != QW_OK:
        raise QWBatchError(rc, qw_batch_last_error(b))


def _instances(inst):
    arr = (qw_instance * len(inst))(*inst)
    return arr


def qw_batch_layout(inst):
    """(offsets, state_bytes, ws_bytes) for a list of qw_instance."""
    n = len(inst)
    arr = _instances(inst)
    offs = (ctypes.c_int64 * max(n, 1))()
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _bcheck(lib().qw_batch_layout(arr, n, offs, ctypes.byref(sb), ctypes.byref(wb)))
    return [int(v) for v in offs[:n]], sb.value, wb.value


def qw_batch_init(inst, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    arr = _instances(inst)
    _bcheck(lib().qw_batch_init(ctypes.byref(h), arr, len(inst), ctypes.c_void_p(workspace_ptr), ws_bytes,
                                ctypes.c_void_p(stream)))
    return h.value


def qw_batch_init_packets(b: int, psi_ptr: int, packets, stream: int) -> None:
    arr = (qw_packet * len(packets))(*packets)
    _bcheck(lib().qw_batch_init_packets(ctypes.c_void_p(b), ctypes.c_void_p(psi_ptr), arr,
                                        ctypes.c_void_p(stream)), b)


def qw_batch_step_n(b: int, psi_ptr: int, n: int, t0: float, dt: float, stream: int) -> None:
    _bcheck(lib().qw_batch_step_n(ctypes.c_void_p(b), ctypes.c_void_p(psi_ptr), int(n), float(t0), float(dt),
                                  ctypes.c_void_p(stream)), b)


def qw_batch_observables(b: int, psi_ptr: int, specs, stream: int, check: bool = True):
    n = len(specs)
    per = 3 * (2 * specs[0].n_max + 1) + 3
    arr = (qw_obs_spec * n)(*specs)
    out = (ctypes.c_double * (per * n))()
    rc = lib().qw_batch_observables(ctypes.c_void_p(b), ctypes.c_void_p(psi_ptr), arr, out, per * n,
                                    ctypes.c_void_p(stream))
    if check:
        _bcheck(rc, b)
    vals = [float(v) for v in out]
    return rc, [vals[i * per:(i + 1) * per] for i in range(n)]


def qw_batch_schedule(b: int, log2n: int, v: int):
    r = (ctypes.c_int32 * 16)()
    cnt = lib().qw_batch_schedule(ctypes.c_void_p(b), int(log2n), int(v), r, 16)
    if cnt < 0:
        _bcheck(cnt, b)
    return [int(x) for x in r[:cnt]]


def qw_batch_set_schedule(b: int, log2n: int, pass_: int, v: int) -> None:
    _bcheck(lib().qw_batch_set_schedule(ctypes.c_void_p(b), int(log2n), int(pass_), int(v)), b)


def qw_batch_set_launch(b: int, row_wg_per_cu: int, col_wg_per_cu: int, graph_steps: int) -> None:
    _bcheck(lib().qw_batch_set_launch(ctypes.c_void_p(b), int(row_wg_per_cu), int(col_wg_per_cu),
                                      int(graph_steps)), b)


def qw_batch_set_loop(b: int, wg_per_cu: int, wait_limit_s: float = 0.0) -> int:
    """Step loop on (wg_per_cu > 0: grid-wide barriers; QW_LOOP_INSTANCE: one
    workgroup per instance) or off (0); -1 only queries.  Returns how many
    grid-wide step-loop workgroups fit one CU (0: no cooperative launches)."""
    fit = ctypes.c_int32()
    _bcheck(lib().qw_batch_set_loop(ctypes.c_void_p(b), int(wg_per_cu), float(wait_limit_s), ctypes.byref(fit)), b)
    return int(fit.value)


def qw_batch_autotune(b: int, psi_ptr: int, dt: float, reps: int, stream: int, max_rows: int = 256):
    rep = (ctypes.c_double * (4 * max_rows))()
    nr = ctypes.c_int32()
    _bcheck(lib().qw_batch_autotune(ctypes.c_void_p(b), ctypes.c_void_p(psi_ptr), float(dt), int(reps), rep,
                                    4 * max_rows, ctypes.byref(nr), ctypes.c_void_p(stream)), b)
    rows = min(nr.value, max_rows)
    return [tuple(float(v) for v in rep[4 * i:4 * i + 4]) for i in range(rows)]


def qw_batch_kernel_timing(b: int, enable: bool) -> None:
    _bcheck(lib().qw_batch_kernel_timing(ctypes.c_void_p(b), int(bool(enable))), b)


def qw_batch_kernel_times(b: int, stream: int):
    out = (ctypes.c_double * 4)()
    _bcheck(lib().qw_batch_kernel_times(ctypes.c_void_p(b), out, 4, ctypes.c_void_p(stream)), b)
    return [float(v) for v in out]


def qw_batch_last_error(b=None) -> str:
    s = lib().qw_batch_last_error(ctypes.c_void_p(b) if b else None)
    return s.decode() if s else ""


def qw_batch_destroy(b: int) -> None:
    lib().qw_batch_destroy(ctypes.c_void_p(b))


# ---- surrogate network -------------------------------------------------------
def _mcheck(rc: int, h=None):
    if rc != QW_OK:
        raise QWError(rc, qw_mlp_last_error(h))


def _p(x) -> ctypes.c_void_p:
    return ctypes.c_void_p(x)


def qw_mlp_param_count(shape: qw_mlp_shape) -> int:
    n = ctypes.c_int64()
    _mcheck(lib().qw_mlp_param_count(ctypes.byref(shape), ctypes.byref(n)))
    return n.value


def qw_mlp_workspace_bytes(shape: qw_mlp_shape) -> int:
    n = ctypes.c_size_t()
    _mcheck(lib().qw_mlp_workspace_bytes(ctypes.byref(shape), ctypes.byref(n)))
    return n.value


def qw_mlp_init(shape: qw_mlp_shape, shift, scale, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    sh = (ctypes.c_float * shape.n_in)(*[float(v) for v in shift])
    sc = (ctypes.c_float * shape.n_in)(*[float(v) for v in scale])
    _mcheck(lib().qw_mlp_init(ctypes.byref(h), ctypes.byref(shape), sh, sc, _p(workspace_ptr), ws_bytes, _p(stream)))
    return h.value


def qw_mlp_set_params(h: int, params_ptr: int, stream: int) -> None:
    _mcheck(lib().qw_mlp_set_params(_p(h), _p(params_ptr), _p(stream)), h)


def qw_mlp_set_output_map(h: int, shift, scale, n_out: int, stream: int) -> None:
    sh = (ctypes.c_float * n_out)(*[float(v) for v in shift])
    sc = (ctypes.c_float * n_out)(*[float(v) for v in scale])
    _mcheck(lib().qw_mlp_set_output_map(_p(h), sh, sc, _p(stream)), h)


def qw_mlp_set_spread_weights(h: int, w, n_out: int, stream: int) -> None:
    wa = (ctypes.c_float * n_out)(*[float(v) for v in w])
    _mcheck(lib().qw_mlp_set_spread_weights(_p(h), wa, _p(stream)), h)


def qw_mlp_get_params(h: int, params_ptr: int, stream: int) -> None:
    _mcheck(lib().qw_mlp_get_params(_p(h), _p(params_ptr), _p(stream)), h)


def qw_mlp_forward(h: int, x_ptr: int, B: int, y_ptr: int, stream: int) -> None:
    _mcheck(lib().qw_mlp_forward(_p(h), _p(x_ptr), int(B), _p(y_ptr), _p(stream)), h)


def qw_mlp_predict(h: int, x_ptr: int, B: int, mean_ptr: int, spread_ptr: int, stream: int) -> None:
    _mcheck(lib().qw_mlp_predict(_p(h), _p(x_ptr), int(B), _p(mean_ptr), _p(spread_ptr), _p(stream)), h)


def qw_mlp_predict_static(h: int, x_ptr: int, B: int, mean_ptr: int, spread_ptr: int, stream: int) -> None:
    _mcheck(lib().qw_mlp_predict_static(_p(h), _p(x_ptr), int(B), _p(mean_ptr), _p(spread_ptr), _p(stream)), h)


def qw_mlp_gradients(h: int, x_ptr: int, t_ptr: int, B: int, grads_ptr, loss_ptr, stream: int) -> None:
    _mcheck(lib().qw_mlp_gradients(_p(h), _p(x_ptr), _p(t_ptr), int(B), _p(grads_ptr), _p(loss_ptr), _p(stream)), h)


def qw_mlp_train_step(h: int, x_ptr: int, t_ptr: int, B: int, lr: float, loss_ptr, stream: int) -> None:
    _mcheck(lib().qw_mlp_train_step(_p(h), _p(x_ptr), _p(t_ptr), int(B), float(lr), _p(loss_ptr), _p(stream)), h)


def qw_gemm_bf16_nt(a_ptr: int, lda: int, b_ptr: int, ldb: int, c_ptr: int, ldc: int, M: int, N: int, K: int,
                    stream: int) -> None:
    _mcheck(lib().qw_gemm_bf16_nt(_p(a_ptr), lda, _p(b_ptr), ldb, _p(c_ptr), ldc, M, N, K, _p(stream)))


def qw_mlp_last_error(h=None) -> str:
    s = lib().qw_mlp_last_error(_p(h) if h else None)
    return s.decode() if s else ""


def qw_mlp_destroy(h: int) -> None:
    lib().qw_mlp_destroy(_p(h))


# ---- convenience owner of device tensors ---------------------------------
def unpack_observables(out, n_max: int) -> dict:
    nb = 2 * n_max + 1
    return {"norm": out[0], "P": list(out[1:1 + nb]), "Pp": list(out[1 + nb:1 + 2 * nb]),
            "Pm": list(out[1 + 2 * nb:1 + 3 * nb]), "P_flip": out[1 + 3 * nb], "P_neg": out[2 + 3 * nb]}


class Sim:
    """State and workspace tensors for one grid on one device, plus its context.

    grid/beam/packet/obs are the dataclasses of ``workloads`` (or anything with
    the same fields).  ``psi`` is a (ny, nx, 4) complex64/complex128 tensor.
    """

    def __init__(self, grid, precision: int = QW_F64, device: str = "cuda:0", beam=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.g = qw_grid(grid.nx, grid.ny, grid.x_min, grid.y_min, grid.lx, grid.ly, grid.c, precision)
        self.dtype = torch.complex64 if precision == QW_F32 else torch.complex128
        nbytes = qw_workspace_bytes(self.g)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.psi = torch.zeros((grid.ny, grid.nx, 4), dtype=self.dtype, device=self.device)
        self.ctx = qw_init_grid(self.g, self.ws.data_ptr(), nbytes, self.stream())
        if beam is not None:
            self.set_beam(beam)

    def stream(self) -> int:
        with self.torch.cuda.device(self.device):
            return self.torch.cuda.current_stream().cuda_stream

    def set_beam(self, b) -> None:
        qw_set_beam(self.ctx, qw_beam(b.mode, b.a0, b.lambda_l, b.w0, b.ramp_periods, b.longitudinal, b.ux, b.uy))

    def set_frame(self, vy: float = 0.0, a_m: float = 0.0) -> None:
        qw_set_frame(self.ctx, qw_frame(vy, a_m))

    def init_packet(self, p) -> None:
        qw_init_packet(self.ctx, self.psi.data_ptr(),
                       qw_packet(p.p0x, p.p0y, p.x0, p.y0, p.sigma_x, p.spin), self.stream())

    def load(self, psi_host) -> None:
        """Copy a (ny, nx, 4) host array into the device state."""
        t = self.torch.as_tensor(psi_host).to(self.dtype)
        self.psi.copy_(t.to(self.device))

    def step(self, n: int, t0: float, dt: float) -> None:
        qw_step_n(self.ctx, self.psi.data_ptr(), n, t0, dt, self.stream())

    def observables(self, o, check: bool = True):
        spec = qw_obs_spec(o.band_ref_idx, o.band_half_idx, o.window_idx, o.n_max, o.spin0)
        rc, out = qw_observables(self.ctx, self.psi.data_ptr(), spec, self.stream(), check=check)
        return out if check else (rc, out)

    def momentum_maps(self):
        """(|phi|^2, |c+|^2, |c-|^2) per momentum cell as a (ny, nx, 3) numpy array, transform order."""
        out = self.torch.empty((self.g.ny, self.g.nx, 3), dtype=self.torch.float64, device=self.device)
        qw_momentum_maps(self.ctx, self.psi.data_ptr(), out.data_ptr(), out.numel(), self.stream())
        self.torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def state(self):
        """Host copy of psi as a numpy complex128 array."""
        self.torch.cuda.synchronize(self.device)
        return self.psi.detach().cpu().to(self.torch.complex128).numpy()

    def close(self) -> None:
        if self.ctx:
            qw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _grid_struct(grid, precision: int) -> qw_grid:
    return qw_grid(grid.nx, grid.ny, grid.x_min, grid.y_min, grid.lx, grid.ly, grid.c, precision)


def _beam_struct(b) -> qw_beam:
    return qw_beam(b.mode, b.a0, b.lambda_l, b.w0, b.ramp_periods, b.longitudinal, b.ux, b.uy)


class Batch:
    """Batch state and workspace tensors on one device, plus the batch handle.

    instances: a list of (grid, beam) pairs (the dataclasses of ``workloads``);
    all instances share ``precision``.  ``psi`` is one uint8 tensor holding
    every instance's state at its offset; ``state(i)`` copies one out.
    """

    def __init__(self, instances, precision: int = QW_F32, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.grids = [g for g, _ in instances]
        self.inst = [qw_instance(_grid_struct(g, precision), _beam_struct(b)) for g, b in instances]
        self.offsets, self.state_bytes, ws_bytes = qw_batch_layout(self.inst)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self.psi = torch.zeros(self.state_bytes, dtype=torch.uint8, device=self.device)
        self.b = qw_batch_init(self.inst, self.ws.data_ptr(), ws_bytes, self.stream())
        self.cdtype = torch.complex64 if precision == QW_F32 else torch.complex128

    def __len__(self):
        return len(self.inst)

    def stream(self) -> int:
        with self.torch.cuda.device(self.device):
            return self.torch.cuda.current_stream().cuda_stream

    def init_packets(self, packets) -> None:
        qw_batch_init_packets(self.b, self.psi.data_ptr(),
                              [qw_packet(p.p0x, p.p0y, p.x0, p.y0, p.sigma_x, p.spin) for p in packets],
                              self.stream())

    def step(self, n: int, t0: float, dt: float) -> None:
        qw_batch_step_n(self.b, self.psi.data_ptr(), n, t0, dt, self.stream())

    def observables(self, specs, check: bool = True):
        s = [qw_obs_spec(o.band_ref_idx, o.band_half_idx, o.window_idx, o.n_max, o.spin0) for o in specs]
        rc, out = qw_batch_observables(self.b, self.psi.data_ptr(), s, self.stream(), check=check)
        return out if check else (rc, out)

    def view(self, i: int):
        """Device tensor view (ny, nx, 4) of instance i's state."""
        g = self.grids[i]
        esize = 8 if self.precision == QW_F32 else 16
        nbytes = g.nx * g.ny * 4 * esize
        raw = self.psi[self.offsets[i]:self.offsets[i] + nbytes]
        return raw.view(self.cdtype).view(g.ny, g.nx, 4)

    def state(self, i: int):
        """Host copy of instance i's psi as a numpy complex128 array."""
        self.torch.cuda.synchronize(self.device)
        return self.view(i).detach().cpu().to(self.torch.complex128).numpy()

    def load(self, i: int, psi_host) -> None:
        self.view(i).copy_(self.torch.as_tensor(psi_host).to(self.cdtype).to(self.device))

    def schedule(self, log2n: int, v: int):
        return qw_batch_schedule(self.b, log2n, v)

    def set_schedule(self, log2n: int, pass_: int, v: int) -> None:
        qw_batch_set_schedule(self.b, log2n, pass_, v)

    def set_launch(self, row_wg_per_cu: int = 0, col_wg_per_cu: int = 0, graph_steps: int = 64) -> None:
        qw_batch_set_launch(self.b, row_wg_per_cu, col_wg_per_cu, graph_steps)

    def set_loop(self, wg_per_cu: int, wait_limit_s: float = 0.0) -> int:
        return qw_batch_set_loop(self.b, wg_per_cu, wait_limit_s)

    def autotune(self, dt: float, reps: int = 20):
        return qw_batch_autotune(self.b, self.psi.data_ptr(), dt, reps, self.stream())

    def close(self) -> None:
        if self.b:
            qw_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Surrogate network ensemble on one device: workspace and parameter tensors
    plus the handle.  x, t, outputs are torch tensors on the same device."""

    def __init__(self, n_in=5, width=256, depth=4, n_out=6, n_nets=4, max_batch=4096, shift=None, scale=None,
                 device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = qw_mlp_shape(n_in, width, depth, n_out, n_nets, max_batch)
        self.per_net = qw_mlp_param_count(self.shape)
        nbytes = qw_mlp_workspace_bytes(self.shape)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        shift = [0.0] * n_in if shift is None else list(shift)
        scale = [1.0] * n_in if scale is None else list(scale)
        self.h = qw_mlp_init(self.shape, shift, scale, self.ws.data_ptr(), nbytes, self.stream())

    def stream(self) -> int:
        with self.torch.cuda.device(self.device):
            return self.torch.cuda.current_stream().cuda_stream

    def _f32(self, a):
        t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device)
        return t.contiguous()

    def set_params(self, flat) -> None:
        """flat: n_nets x per_net values (host or device)."""
        p = self._f32(flat).reshape(-1)
        assert p.numel() == self.shape.n_nets * self.per_net
        qw_mlp_set_params(self.h, p.data_ptr(), self.stream())
        self.torch.cuda.synchronize(self.device)

    def set_output_map(self, shift, scale) -> None:
        qw_mlp_set_output_map(self.h, shift, scale, self.shape.n_out, self.stream())

    def set_spread_weights(self, w) -> None:
        """Per-output weights of the ensemble spread predict() returns (default all one)."""
        qw_mlp_set_spread_weights(self.h, w, self.shape.n_out, self.stream())

    def params(self):
        out = self.torch.empty(self.shape.n_nets * self.per_net, dtype=self.torch.float32, device=self.device)
        qw_mlp_get_params(self.h, out.data_ptr(), self.stream())
        return out.view(self.shape.n_nets, self.per_net)

    def forward(self, x):
        x = self._f32(x)
        B = x.shape[0]
        y = self.torch.empty((self.shape.n_nets, B, self.shape.n_out), dtype=self.torch.float32, device=self.device)
        qw_mlp_forward(self.h, x.data_ptr(), B, y.data_ptr(), self.stream())
        return y

    def predict(self, x):
        x = self._f32(x)
        B = x.shape[0]
        mean = self.torch.empty((B, self.shape.n_out), dtype=self.torch.float32, device=self.device)
        spread = self.torch.empty(B, dtype=self.torch.float32, device=self.device)
        qw_mlp_predict(self.h, x.data_ptr(), B, mean.data_ptr(), spread.data_ptr(), self.stream())
        return mean, spread

    def gradients(self, x, t):
        x, t = self._f32(x), self._f32(t)
        g = self.torch.empty((self.shape.n_nets, self.per_net), dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(self.shape.n_nets, dtype=self.torch.float32, device=self.device)
        qw_mlp_gradients(self.h, x.data_ptr(), t.data_ptr(), x.shape[0], g.data_ptr(), loss.data_ptr(),
                         self.stream())
        return g, loss

    def train_step(self, x, t, lr: float, loss=None):
        """x, t: device float32 tensors (contiguous); loss: optional [n_nets] device tensor."""
        qw_mlp_train_step(self.h, x.data_ptr(), t.data_ptr(), x.shape[0], lr,
                          None if loss is None else loss.data_ptr(), self.stream())

    def close(self) -> None:
        if self.h:
            qw_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
