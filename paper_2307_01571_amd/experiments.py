"""Paper-fidelity runs of the full model (Sec. II.D, III and IV) on the
library: the full Gaussian-beam standing wave, the box co-moving with the
electron and the gauge shift A_m, at the paper's parameters.

Units: atomic units with hbar = m = 1, so the paper's m c is C_AU and its
hbar k_L = 0.1 m c is k_L = 0.1 C_AU.  Parameters of the showcase (Sec. II.D):
a 2048 x 128 grid over 80 lambda x 40 lambda, x in [-40, 40) lambda, the y
window starting at [-160, -120) lambda and moving with v_y = c/sqrt2; packet
at kinetic p0 = (-hbar k_L, m c), r0 = (140 lambda_C, -140 lambda),
sigma_p = hbar k_L/200, spin +x; dt = 0.05 hbar/(m c^2) and the travel time
280 lambda sqrt2 / c; omega = c k_L, A0 = 0.1 m c/q, eps = 0.02, A_m = m c.

* ``showcase`` (E1): band and spin-resolved probabilities, and the
  spin-resolved densities |c^+-(p)|^2 at the diffracted peak p = (hbar k_L,
  m c) (the paper reports 4.6e-5 and 3.9e-3 there; its values are grid-point
  densities of an unstated normalisation, so the comparison is the ratio).
* ``scaling`` (E3): the spin-flip density at the diffracted peak over
  eps in {0.01, 0.02, 0.05, 0.1} and hbar k_L/(m c) in {0.05, 0.07, 0.1};
  the paper finds it proportional to (k_L/eps)^2.
* ``longitudinal`` (E4): with and without A_x; the paper finds the
  difference of |c^s|^2 proportional to eps^2, nearly independent of k_L.
* ``diffraction`` (E5, E6): eps = 0.1, k_L = 0.1, A0 = 0.4 m c/q on
  2048 x 256 at p_x = -hbar k_L and p_x = 0: the momentum of the peak of each
  diffraction order against the energy-conservation estimate of Eq. 22,
  Delta p_y = -2 n hbar k_L p_x/(m c) - 2 n^2 hbar^2 k_L^2/(m c).

    python -m paper_2307_01571_amd.experiments showcase --out e1.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import qw
from . import workloads as W

C = W.C_AU


def _log(*a):
    print("[experiments]", *a, file=sys.stderr, flush=True)


def setup(kl_mc=0.1, eps=0.02, a0_mc=0.1, nx=2048, ny=128, box_x=80, box_y=40, px_kl=-1.0, longitudinal=1,
          w0_kl_mc=None, sigma_p_mc=None):
    """Grid, beam, packet, frame and step plan of the showcase family (lengths in lambda).

    By default every length follows lambda: the box, the start y0 = -140
    lambda and the travel time, the waist w0 = 1/(k_L eps) and the packet's
    sigma_p = hbar k_L/200.  w0_kl_mc fixes the waist at 1/(k eps) with k =
    w0_kl_mc m c/hbar whatever k_L; sigma_p_mc fixes sigma_p in m c."""
    kl = kl_mc * C
    lam = 2 * math.pi / kl
    lam_c = 2 * math.pi / C
    g = W.GridSpec(nx=nx, ny=ny, x_min=-box_x / 2 * lam, y_min=(-140 - box_y / 2) * lam, lx=box_x * lam,
                   ly=box_y * lam)
    k_w0 = kl if w0_kl_mc is None else w0_kl_mc * C
    b = W.BeamSpec(mode=qw.QW_BEAM_GAUSSIAN_FULL, a0=a0_mc * C, lambda_l=lam, w0=1.0 / (k_w0 * eps), ramp_periods=0.0,
                   longitudinal=longitudinal)
    sigma_p = kl / 200 if sigma_p_mc is None else sigma_p_mc * C
    p = W.PacketSpec(p0x=px_kl * kl, p0y=C, x0=140 * lam_c, y0=-140 * lam, sigma_x=1 / (2 * sigma_p), spin=1)
    dt = 0.05 / C ** 2
    steps = int(round(280 * lam * math.sqrt(2) / C / dt))
    half = box_x  # k_L / dk_x with dk_x = 2 pi / (box_x lambda)
    o = W.ObsSpec(band_ref_idx=int(round(px_kl * half)), band_half_idx=half, window_idx=half // 2, n_max=3, spin0=1)
    return dict(grid=g, beam=b, packet=p, obs=o, vy=C / math.sqrt(2), a_m=C, dt=dt, steps=steps, kl=kl, lam=lam)


def run(cfg, prec=qw.QW_F64, chunk=50_000):
    """Propagate to the end; returns observables, momentum maps and timing."""
    sim = qw.Sim(cfg["grid"], prec, beam=cfg["beam"])
    sim.set_frame(cfg["vy"], cfg["a_m"])
    sim.init_packet(cfg["packet"])
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < cfg["steps"]:
        n = min(chunk, cfg["steps"] - done)
        sim.step(n, done * cfg["dt"], cfg["dt"])
        done += n
        torch.cuda.synchronize()
        _log(f"  {done}/{cfg['steps']} steps, {time.perf_counter() - t0:.1f} s")
    el = time.perf_counter() - t0
    obs = qw.unpack_observables(sim.observables(cfg["obs"]), cfg["obs"].n_max)
    maps = sim.momentum_maps()
    sim.close()
    return obs, maps, el


def run_many(cfgs, prec=qw.QW_F64, chunk=20_000):
    """Several runs at once, each on its own stream (default priority): one
    2048 x 128 run fills about half the GPU, so concurrent runs overlap.
    Returns [(observables, momentum maps, seconds of the whole group)]."""
    import torch
    sims, streams = [], []
    for cfg in cfgs:
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            sim = qw.Sim(cfg["grid"], prec, beam=cfg["beam"])
            sim.set_frame(cfg["vy"], cfg["a_m"])
            sim.init_packet(cfg["packet"])
        sims.append(sim)
        streams.append(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = [0] * len(cfgs)
    while any(d < c["steps"] for d, c in zip(done, cfgs)):
        for i, (sim, st, cfg) in enumerate(zip(sims, streams, cfgs)):
            if done[i] >= cfg["steps"]:
                continue
            n = min(chunk, cfg["steps"] - done[i])
            with torch.cuda.stream(st):
                sim.step(n, done[i] * cfg["dt"], cfg["dt"])
            done[i] += n
        torch.cuda.synchronize()
        _log(f"  {min(done)}..{max(done)} steps of {len(cfgs)} runs, {time.perf_counter() - t0:.1f} s")
    el = time.perf_counter() - t0
    out = []
    for sim, st, cfg in zip(sims, streams, cfgs):
        with torch.cuda.stream(st):
            obs = qw.unpack_observables(sim.observables(cfg["obs"]), cfg["obs"].n_max)
            maps = sim.momentum_maps()
        sim.close()
        out.append((obs, maps, el))
    return out


def momenta(cfg):
    g = cfg["grid"]
    px = 2 * math.pi * np.fft.fftfreq(g.nx, d=g.lx / g.nx)
    py = 2 * math.pi * np.fft.fftfreq(g.ny, d=g.ly / g.ny) + cfg["a_m"]  # kinetic
    return px, py


def peak_near(cfg, maps, px_target, py_target, col=0, radius=(3, 6)):
    """Largest value of maps[..., col] within a few cells of (px, py) (kinetic)."""
    px, py = momenta(cfg)
    ix = int(np.argmin(np.abs(px - px_target)))
    iy = int(np.argmin(np.abs(py - py_target)))
    best, at = -1.0, (iy, ix)
    for dy in range(-radius[1], radius[1] + 1):
        for dx in range(-radius[0], radius[0] + 1):
            j, i = (iy + dy) % len(py), (ix + dx) % len(px)
            if maps[j, i, col] > best:
                best, at = maps[j, i, col], (j, i)
    return float(best), float(px[at[1]]), float(py[at[0]])


def showcase(prec=qw.QW_F64, **kw):
    cfg = setup(**kw)
    _log(f"showcase: {cfg['grid'].nx}x{cfg['grid'].ny}, {cfg['steps']} steps")
    obs, maps, el = run(cfg, prec)
    total = float(np.sum(maps[..., 0]))
    # the diffracted peak p = (+hbar k_L, m c); normalise densities to the total
    cp, cpx, cpy = peak_near(cfg, maps, cfg["kl"], C, col=1)
    cm, _, _ = peak_near(cfg, maps, cfg["kl"], C, col=2)
    c0p, _, _ = peak_near(cfg, maps, -cfg["kl"], C, col=1)
    return {"config": {"kl_mc": cfg["kl"] / C, "grid": [cfg["grid"].nx, cfg["grid"].ny], "steps": cfg["steps"],
                       "dt": cfg["dt"], "eps": 1 / (cfg["kl"] * cfg["beam"].w0), "a0": cfg["beam"].a0,
                       "prec": "f64" if prec == qw.QW_F64 else "f32"},
            "seconds": el, "cell_steps_per_s": cfg["grid"].nx * cfg["grid"].ny * cfg["steps"] / el,
            "bands": {k: (list(map(float, v)) if isinstance(v, np.ndarray) else v) for k, v in obs.items()},
            "peak_plus_k": {"c_plus_sq": cp / total, "c_minus_sq": cm / total, "ratio_minus_over_plus": cm / cp,
                            "at": [cpx / cfg["kl"], cpy / C]},
            "peak_minus_k_c_plus_sq": c0p / total}


# Readings of the scan's parameters (which lengths follow lambda = 2 pi/k_L):
#   scaled      every length follows lambda (box, y0, travel time, w0 = 1/(k_L eps), sigma_p = hbar k_L/200)
#   fixed_w0    as scaled, but w0 = 1/(k eps) with k = 0.1 m c/hbar for every k_L
#   fixed_sigma as scaled, but sigma_p = 0.1 m c/200 for every k_L
READINGS = {"scaled": {}, "fixed_w0": {"w0_kl_mc": 0.1}, "fixed_sigma": {"sigma_p_mc": 0.1 / 200}}


def scaling(prec=qw.QW_F32, eps_list=(0.01, 0.02, 0.05, 0.1), kl_list=(0.05, 0.07, 0.1), longitudinal_off=False,
            reading="scaled"):
    """The scan's runs of one k_L go together (equal step counts).  Each row
    has the spin-flip density at the diffracted peak as a share of the total
    (c_minus_sq) and the areas of one grid cell in momentum and position
    space, which turn the share into other normalisations of |phi|^2."""
    rows = []
    extra = READINGS[reading]
    for kl in kl_list:
        cfgs, keys = [], []
        for eps in eps_list:
            for lon in ((1, 0) if longitudinal_off else (1,)):
                cfgs.append(setup(kl_mc=kl, eps=eps, longitudinal=lon, **extra))
                keys.append((eps, lon))
        _log(f"scaling: k_L = {kl} m c, {len(cfgs)} runs of {cfgs[0]['steps']} steps")
        for (eps, lon), cfg, (obs, maps, el) in zip(keys, cfgs, run_many(cfgs, prec)):
            total = float(np.sum(maps[..., 0]))
            cp, _, _ = peak_near(cfg, maps, cfg["kl"], C, col=1)
            cm, _, _ = peak_near(cfg, maps, cfg["kl"], C, col=2)
            g = cfg["grid"]
            rows.append({"reading": reading, "kl_mc": kl, "eps": eps, "longitudinal": lon, "steps": cfg["steps"],
                         "group_seconds": el, "w0": cfg["beam"].w0, "sigma_x": cfg["packet"].sigma_x,
                         "cell_area_p": (2 * math.pi) ** 2 / (g.lx * g.ly), "cell_area_r": g.lx * g.ly / (g.nx * g.ny),
                         "cells": g.nx * g.ny,
                         "c_plus_sq": cp / total, "c_minus_sq": cm / total,
                         "P_plus1": float(obs["P"][cfg["obs"].n_max + 1]),
                         "P_plus1_plus": float(obs["Pp"][cfg["obs"].n_max + 1]),
                         "P_plus1_flip": float(obs["Pm"][cfg["obs"].n_max + 1]), "P_flip": obs["P_flip"]})
    return rows


def loglog_slope(x, y):
    x, y = np.log(np.asarray(x, float)), np.log(np.asarray(y, float))
    return float(np.polyfit(x, y, 1)[0])


def diffraction(prec=qw.QW_F64, px_kl=-1.0, n_orders=(-3, -2, -1, 0, 1, 2, 3)):
    cfg = setup(kl_mc=0.1, eps=0.1, a0_mc=0.4, ny=256, px_kl=px_kl)
    _log(f"diffraction: p_x = {px_kl} hbar k_L, {cfg['steps']} steps")
    obs, maps, el = run(cfg, prec)
    px, py = momenta(cfg)
    kl = cfg["kl"]
    total = float(np.sum(maps[..., 0]))
    rows = []
    o = cfg["obs"]
    dkx = 2 * math.pi / cfg["grid"].lx
    for n in n_orders:
        pxn = px_kl * kl + 2 * n * kl
        ix = int(np.argmin(np.abs(px - pxn)))
        col = maps[:, ix, 0]
        j = int(np.argmax(col))
        dpy = float(py[j] - C)
        est = -2 * n * kl * (px_kl * kl) / C - 2 * n * n * kl * kl / C
        # the largest density anywhere in the order's window of columns
        cols = np.nonzero(np.abs(np.rint((px - pxn) / dkx)) <= o.window_idx)[0]
        sub = maps[:, cols, 0]
        jj, ii = np.unravel_index(int(np.argmax(sub)), sub.shape)
        pop = float(obs["P"][o.n_max + n]) if abs(n) <= o.n_max else None
        # the local maxima of |c+|^2 and |c-|^2 around the Eq. 22 location
        # (p_x0 + 2 n hbar k_L, m c + Delta p_y): within 10 cells in p_x and
        # 8 cells in p_y, as the largest value of each projection at the peak
        iy22 = int(np.argmin(np.abs(py - (C + est))))
        near_x = [(ix + d) % len(px) for d in range(-10, 11)]
        near_y = [(iy22 + d) % len(py) for d in range(-8, 9)]
        box = maps[np.ix_(near_y, near_x)]
        rows.append({"n": n, "band_P": pop, "peak_density": float(col[j]) / total, "dpy_measured": dpy,
                     "dpy_eq22": est, "dpy_cell": float(2 * math.pi / cfg["grid"].ly),
                     "window_peak_density": float(sub[jj, ii]) / total,
                     "window_peak_at": [float(px[cols[ii]] / kl), float((py[jj] - C) / kl)],
                     "c_plus_sq": float(maps[j, ix, 1]) / total, "c_minus_sq": float(maps[j, ix, 2]) / total,
                     "c_plus_sq_localmax": float(box[..., 1].max()) / total,
                     "c_minus_sq_localmax": float(box[..., 2].max()) / total})
    return {"px_kl": px_kl, "seconds": el, "orders": rows,
            "bands": {k: (list(map(float, v)) if isinstance(v, np.ndarray) else v) for k, v in obs.items()}}


def drift(kl_mc=0.1, eps=0.02, checkpoints=10, chunk=10_000):
    """FP32 against FP64 along one run of the scan's family (Sec. IV.B
    set-up), both propagated side by side on their own streams: at
    `checkpoints` evenly spaced step counts, the spin-flip density at the
    diffracted peak, P_+1, P_flip and the norm of each, and the FP32
    relative errors.  The growth of those errors with the step count (the
    log-log slope over the later checkpoints) tells a systematic per-step
    bias (slope 1) from accumulated rounding (slope 1/2)."""
    import torch
    cfg = setup(kl_mc=kl_mc, eps=eps)
    total_steps = cfg["steps"]
    marks = [int(round(total_steps * (i + 1) / checkpoints)) for i in range(checkpoints)]
    sims, streams = {}, {}
    for name, prec in (("f32", qw.QW_F32), ("f64", qw.QW_F64)):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            sim = qw.Sim(cfg["grid"], prec, beam=cfg["beam"])
            sim.set_frame(cfg["vy"], cfg["a_m"])
            sim.init_packet(cfg["packet"])
        sims[name], streams[name] = sim, st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, rows = 0, []
    n_max = cfg["obs"].n_max
    for mark in marks:
        while done < mark:
            n = min(chunk, mark - done)
            for name in sims:
                with torch.cuda.stream(streams[name]):
                    sims[name].step(n, done * cfg["dt"], cfg["dt"])
            done += n
            torch.cuda.synchronize()
        row = {"steps": done}
        for name in sims:
            with torch.cuda.stream(streams[name]):
                obs = qw.unpack_observables(sims[name].observables(cfg["obs"]), n_max)
                maps = sims[name].momentum_maps()
            total = float(np.sum(maps[..., 0]))
            cm, _, _ = peak_near(cfg, maps, cfg["kl"], C, col=2)
            row[name] = {"c_minus_sq": cm / total, "P_plus1": float(obs["P"][n_max + 1]), "P_flip": obs["P_flip"],
                         "norm": obs["norm"]}
        row["rel_err"] = {k: abs(row["f32"][k] - row["f64"][k]) / abs(row["f64"][k])
                          for k in ("c_minus_sq", "P_plus1", "P_flip")}
        row["norm_diff"] = row["f32"]["norm"] - row["f64"]["norm"]
        rows.append(row)
        _log(f"  drift: {done}/{total_steps} steps, {time.perf_counter() - t0:.1f} s, rel err {row['rel_err']}")
    for sim in sims.values():
        sim.close()
    late = rows[len(rows) // 2:]
    slopes = {k: loglog_slope([r["steps"] for r in late], [r["rel_err"][k] for r in late])
              for k in ("c_minus_sq", "P_plus1", "P_flip")}
    return {"config": {"kl_mc": kl_mc, "eps": eps, "grid": [cfg["grid"].nx, cfg["grid"].ny], "dt": cfg["dt"],
                       "steps": total_steps}, "rows": rows, "loglog_slope_late_half": slopes}


def _density_breakdown(cfg, maps):
    """Sums of |phi|^2, |c+|^2, |c-|^2 and of the rest (negative energy) over
    the momentum cells near the incoming packet (p_x = -k_L), near the +1
    order (p_x = +k_L) and over all other cells."""
    px, _ = momenta(cfg)
    kl = cfg["kl"]
    near_m = np.abs(px + kl) < kl / 2
    near_p = np.abs(px - kl) < kl / 2
    rest = ~(near_m | near_p)
    comp = {"all": maps[..., 0], "c_plus": maps[..., 1], "c_minus": maps[..., 2],
            "neg": maps[..., 0] - maps[..., 1] - maps[..., 2]}
    return {f"{r}/{c}": float(np.sum(v[:, m])) for r, m in (("-1", near_m), ("+1", near_p), ("rest", rest))
            for c, v in comp.items()}


def drift_split(kl_mc=0.1, eps=0.02, split=0.5, checkpoints=5, chunk=10_000):
    """FP64 through the first part of one run of the scan family (the share
    split of its steps), then FP32 and FP64 continued from that same state
    to the end, once with the field and once without it (QW_BEAM_NONE), all
    four side by side on their own streams.  The growth of the FP32 relative
    errors of P_+1 and of the flip density at the peak with and without the
    field tells the free-flight operators (transforms, kinetic step) from the
    interaction step as the source of FP32 drift; the breakdown of the
    densities by momentum region and energy sign, at the first and the last
    checkpoint, tells where the FP32 norm grows."""
    import torch
    cfg = setup(kl_mc=kl_mc, eps=eps)
    total = cfg["steps"]
    half = int(round(total * split))
    base = qw.Sim(cfg["grid"], qw.QW_F64, beam=cfg["beam"])
    base.set_frame(cfg["vy"], cfg["a_m"])
    base.init_packet(cfg["packet"])
    done = 0
    while done < half:
        n = min(chunk * 5, half - done)
        base.step(n, done * cfg["dt"], cfg["dt"])
        done += n
        torch.cuda.synchronize()
        _log(f"  drift_split: FP64 to the split, {done}/{half} steps")
    state = base.psi.clone()
    base.close()
    off = W.BeamSpec(mode=qw.QW_BEAM_NONE)
    runs = {}
    for field, beam in (("on", cfg["beam"]), ("off", off)):
        for name, prec in (("f32", qw.QW_F32), ("f64", qw.QW_F64)):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                sim = qw.Sim(cfg["grid"], prec, beam=beam)
                sim.set_frame(cfg["vy"], cfg["a_m"])
                sim.psi.copy_(state.to(sim.psi.dtype))
            runs[(field, name)] = (sim, st)
    torch.cuda.synchronize()
    marks = [half + int(round((total - half) * (i + 1) / checkpoints)) for i in range(checkpoints)]
    n_max = cfg["obs"].n_max
    rows, parts = [], {}
    for mark in marks:
        while done < mark:
            n = min(chunk, mark - done)
            for sim, st in runs.values():
                with torch.cuda.stream(st):
                    sim.step(n, done * cfg["dt"], cfg["dt"])
            done += n
            torch.cuda.synchronize()
        row = {"steps": done, "after_split": done - half}
        vals = {}
        for key, (sim, st) in runs.items():
            with torch.cuda.stream(st):
                obs = qw.unpack_observables(sim.observables(cfg["obs"]), n_max)
                maps = sim.momentum_maps()
            tot = float(np.sum(maps[..., 0]))
            cm, _, _ = peak_near(cfg, maps, cfg["kl"], C, col=2)
            vals[key] = {"P_plus1": float(obs["P"][n_max + 1]), "c_minus_sq": cm / tot, "norm": obs["norm"]}
            if mark in (marks[0], marks[-1]):
                parts.setdefault(key, []).append(_density_breakdown(cfg, maps))
        for field in ("on", "off"):
            a, b = vals[(field, "f32")], vals[(field, "f64")]
            row[field] = {k: abs(a[k] - b[k]) / abs(b[k]) for k in ("P_plus1", "c_minus_sq")}
            row[field]["norm_diff"] = a["norm"] - b["norm"]
            row[field]["P_plus1_f64"] = b["P_plus1"]
            row[field]["c_minus_sq_f64"] = b["c_minus_sq"]
        rows.append(row)
        _log(f"  drift_split: {done}/{total} steps, on {row['on']}, off {row['off']}")
    for sim, _ in runs.values():
        sim.close()
    # per region and component: FP32's relative change between the first and
    # the last checkpoint minus FP64's, and FP64's share of the total at the end
    growth = {}
    for field in ("on", "off"):
        (f32a, f32b), (f64a, f64b) = parts[(field, "f32")], parts[(field, "f64")]
        tot = f64b["-1/all"] + f64b["+1/all"] + f64b["rest/all"]
        growth[field] = {k: {"share_f64": f64b[k] / tot,
                             "excess_rel_growth": (f32b[k] / f32a[k] - f64b[k] / f64a[k]) if f32a[k] > 0 and f64a[k] > 0 else None,
                             "excess_abs_growth": (f32b[k] - f32a[k]) - (f64b[k] - f64a[k])}
                         for k in f64b}
    return {"config": {"kl_mc": kl_mc, "eps": eps, "grid": [cfg["grid"].nx, cfg["grid"].ny], "steps": total,
                       "split": half}, "rows": rows, "growth_first_to_last_checkpoint": growth}


def bin_gains(kl_mc=0.1, eps=0.02, bins=(-240, -160, -80, -1, 0, 1, 80, 160, 240), steps=40_000):
    """Norm gain per step of single momentum cells under the free step of
    the scan family's grid and frame (field off): a plane wave at (kx, ky =
    0) with one unit spinor component, propagated steps steps in FP32 and in
    FP64; returns log(norm after / norm before) / steps per bin and
    component.  The step's gain for one cell, whatever the other cells
    hold, measured on the kernels themselves."""
    import torch
    cfg = setup(kl_mc=kl_mc, eps=eps)
    g = cfg["grid"]
    off = W.BeamSpec(mode=qw.QW_BEAM_NONE)
    ix = torch.arange(g.nx, dtype=torch.float64, device="cuda")
    out = {}
    for name, prec in (("f32", qw.QW_F32), ("f64", qw.QW_F64)):
        rows = {}
        for kx in bins:
            gains = []
            for comp in range(4):
                sim = qw.Sim(g, prec, beam=off)
                sim.set_frame(cfg["vy"], cfg["a_m"])
                w = torch.zeros((g.ny, g.nx, 4), dtype=torch.complex128, device="cuda")
                w[:, :, comp] = torch.exp(2j * math.pi * kx * ix / g.nx)[None, :] / math.sqrt(g.nx * g.ny)
                sim.psi.copy_(w.to(sim.psi.dtype))
                n0 = float((sim.psi.to(torch.complex128).abs() ** 2).sum())
                sim.step(steps, 0.0, cfg["dt"])
                torch.cuda.synchronize()
                n1 = float((sim.psi.to(torch.complex128).abs() ** 2).sum())
                sim.close()
                gains.append(math.log(n1 / n0) / steps)
            rows[str(kx)] = gains
            _log(f"  bin_gains {name} kx {kx}: " + " ".join(f"{v:+.3e}" for v in gains))
        out[name] = rows
    return {"config": {"kl_mc": kl_mc, "grid": [g.nx, g.ny], "steps": steps,
                       "transform_gain_x": qw.qw_transform_gain(g.nx, qw.QW_F32)}, "gain_per_step": out}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["showcase", "scaling", "longitudinal", "diffraction", "drift", "drift_split", "bin_gains"])
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--split", type=float, default=0.5, help="drift_split: share of the run propagated in FP64 first")
    ap.add_argument("--out", required=True)
    ap.add_argument("--kl", type=float, nargs="+", default=[0.05, 0.07, 0.1], help="hbar k_L / (m c) of the scans")
    ap.add_argument("--eps", type=float, nargs="+", default=[0.01, 0.02, 0.05, 0.1], help="beam divergences of the scans")
    ap.add_argument("--reading", choices=sorted(READINGS), default="scaled",
                    help="which lengths of the scans follow the laser wavelength")
    a = ap.parse_args(argv)
    qw.lib()
    prec = qw.QW_F64 if a.prec == "f64" else qw.QW_F32
    if a.what == "showcase":
        res = showcase(prec)
    elif a.what == "scaling":
        rows = scaling(prec, eps_list=a.eps, kl_list=a.kl, reading=a.reading)
        res = {"rows": rows}
        for kl in sorted({r["kl_mc"] for r in rows}):
            sel = [r for r in rows if r["kl_mc"] == kl]
            res[f"slope_vs_eps_kl{kl}"] = loglog_slope([r["eps"] for r in sel], [r["c_minus_sq"] for r in sel])
        for eps in sorted({r["eps"] for r in rows}):
            sel = [r for r in rows if r["eps"] == eps]
            if len(sel) > 1:
                res[f"slope_vs_kl_eps{eps}"] = loglog_slope([r["kl_mc"] for r in sel],
                                                            [r["c_minus_sq"] for r in sel])
    elif a.what == "longitudinal":
        rows = scaling(prec, eps_list=a.eps, kl_list=a.kl, longitudinal_off=True, reading=a.reading)
        res = {"rows": rows}
        for kl in sorted({r["kl_mc"] for r in rows}):
            d = []
            for eps in sorted({r["eps"] for r in rows}):
                on = [r for r in rows if r["kl_mc"] == kl and r["eps"] == eps and r["longitudinal"] == 1][0]
                off = [r for r in rows if r["kl_mc"] == kl and r["eps"] == eps and r["longitudinal"] == 0][0]
                d.append((eps, abs(off["c_minus_sq"] - on["c_minus_sq"]), abs(off["c_plus_sq"] - on["c_plus_sq"])))
            res[f"diff_kl{kl}"] = d
            res[f"slope_minus_kl{kl}"] = loglog_slope([x[0] for x in d], [x[1] for x in d])
            res[f"slope_plus_kl{kl}"] = loglog_slope([x[0] for x in d], [x[2] for x in d])
    elif a.what == "drift":
        res = drift(kl_mc=a.kl[0], eps=a.eps[0])
    elif a.what == "bin_gains":
        res = bin_gains(kl_mc=a.kl[0], eps=a.eps[0])
    elif a.what == "drift_split":
        res = drift_split(kl_mc=a.kl[0], eps=a.eps[0], split=a.split)
    else:
        res = {"E5": diffraction(prec, px_kl=-1.0), "E6": diffraction(prec, px_kl=0.0)}
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    _log(json.dumps(res)[:2000])


if __name__ == "__main__":
    main()
