#!/usr/bin/env python3
"""Throughput of the split-operator step on one MI355X.

One bench step is one full Strang step (row pass + column pass) of the
2048 x 2048 FP32 workload (box 64 lambda, w0 = 16 lambda, A0 = 0.5, Gaussian
packet at p = (-k_L, 0.1 k_L)).  By default the timed region is the whole
5e4-step propagation, run as one qw_step_n call with the state resident in
HBM.  Before it, untimed (this also brings the GPU to its working clocks):
  * a run of --timing-steps steps with per-launch HIP events, giving the
    average duration of each pass and its fraction of the HBM roofline;
  * torch's plain copy of the state, the attainable bandwidth.
Afterwards, untimed:
  * the same propagation in FP64, whose band and spin probabilities the FP32
    result is compared with (absolute errors; relative ones for values above
    the FP32 floor of about 1e-9);
  * the batching workload (96 uneven instances, autotuned): batched and
    one-by-one rates and their ratio;
  * the same step written with torch.fft (rocFFT) and torch elementwise
    ops, and the bare library transforms alone, for comparison;
  * the oracle (FP64 CPU) on a bounded sample of the same workload.
Prints one JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 50000] [--warmup 500]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4  # wave64 VALU issue: CUs x SIMDs x GHz / cycles per instruction
BYTES_PER_CELL_PASS = {"f32": 64, "f64": 128}  # read + write of 4 complex per pass
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_2048sq_f32.json")


# the sources of the row and column pass kernels (device code and launch shapes)
PASS_SOURCES = ("qw_device.hpp", "qw_kernels.inl", "qw_launch.hpp", "qw_kernels_f32.hip", "qw_kernels_f64.hip")


def kernel_source_hash() -> str:
    """Hash of the sources that define the row and column pass kernels.

    Measured traffic is reported only for the kernels it was taken on; the
    other sources (host code, reductions, batched and network kernels) do
    not enter.
    """
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2307_01571_amd", "csrc")
    for name in PASS_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_counters(kernel: str):
    """Counter figures per launch from the committed rocprofv3 runs, if still current.

    Returns {"bytes": HBM read + write bytes, "valu_insts": wave-level VALU
    instructions (None if not recorded)} or None when the kernel sources have
    changed since the counters were taken.
    """
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    return {"bytes": k["read_bytes"] + k["write_bytes"], "valu_insts": k.get("valu_insts")}


# the symbols the traffic record keys: the whole-state launches of the middle
# passes (timed per launch for the roofline) and the per-block launches of the
# two-chain step loop
COUNTER_KERNELS = {
    "col_pass": "void qw::col_pass<float, 2048, 0, 0, false>(qw::ColArgs)",
    "row_pass": "void qw::row_pass<float, 2048, 1, 0, false>(qw::RowArgs)",
    "col_pass_one_block": "void qw::col_pass<float, 2048, 0, 0, true>(qw::ColArgs)",
    "row_pass_one_block": "void qw::row_pass<float, 2048, 1, 0, true>(qw::RowArgs)",
}
SQ_KEYS = {"SQ_WAVES": "waves", "SQ_INSTS_VALU": "valu_insts", "SQ_INSTS_LDS": "lds_insts",
           "SQ_LDS_BANK_CONFLICT": "lds_bank_conflicts", "SQ_WAIT_INST_LDS": "wait_inst_lds",
           "SQ_WAVE_CYCLES": "wave_cycles", "SQ_BUSY_CYCLES": "busy_cycles",
           "SQ_ACTIVE_INST_VALU": "active_inst_valu"}


def read_counter_csvs(d):
    """{kernel name: {counter: mean value per dispatch}} from the
    *counter_collection.csv files of one rocprofv3 --pmc output folder."""
    import csv
    import glob
    sums, counts = {}, {}
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                key = (row["Kernel_Name"], row["Counter_Name"])
                sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
                counts.setdefault(key, set()).add((fn, row.get("Dispatch_Id") or row.get("Correlation_Id")))
    out = {}
    for (k, c), v in sums.items():
        out.setdefault(k, {})[c] = v / len(counts[(k, c)])
    return out


def record_counters(d):
    """Write the traffic record from rocprofv3 --pmc runs kept under d:
    d/fetch (FETCH_SIZE), d/write (WRITE_SIZE) and d/sq (SQ_ counters) of the
    counter command, d/copy_fetch and d/copy_write of --copy-probe.  The KiB
    counters are scaled by the factors that make the copy kernel's read and
    written KiB equal the bytes it moves.  Prints a summary table."""
    fetch, write = read_counter_csvs(os.path.join(d, "fetch")), read_counter_csvs(os.path.join(d, "write"))
    sq = read_counter_csvs(os.path.join(d, "sq")) if os.path.isdir(os.path.join(d, "sq")) else {}
    cf, cw = read_counter_csvs(os.path.join(d, "copy_fetch")), read_counter_csvs(os.path.join(d, "copy_write"))
    copy_kib = 2048 * 2048 * 4 * 8 / 1024  # one 2048^2 FP32 state, read once and written once
    ck = [k for k in cf if "copyBuffer" in k]  # the device-to-device copy (not the fill before it)
    if not ck:
        raise SystemExit("no copy kernel in the copy-probe runs")
    read_scale = copy_kib / cf[ck[0]]["FETCH_SIZE"]
    write_scale = copy_kib / cw[ck[0]]["WRITE_SIZE"]
    rec = {"source_sha256": kernel_source_hash(), "read_scale": read_scale, "write_scale": write_scale,
           "copy_kernel": ck[0],
           "note": "KiB counters scaled by the copy kernel's factors; bytes per launch; SQ_ counters per launch",
           "kernels": {}}
    alg = BYTES_PER_CELL_PASS["f32"] * 2048 * 2048
    print(f"copy kernel {ck[0]}: FETCH_SIZE {cf[ck[0]]['FETCH_SIZE']:.1f} KiB -> read scale {read_scale:.4f}; "
          f"WRITE_SIZE {cw[ck[0]]['WRITE_SIZE']:.1f} KiB -> write scale {write_scale:.4f}")
    print(f"{'kernel':58s} {'FETCH KiB':>10s} {'WRITE KiB':>10s} {'read MiB':>9s} {'write MiB':>9s} "
          f"{'total/alg':>9s}")
    for key, name in COUNTER_KERNELS.items():
        if name not in fetch or name not in write:
            continue
        one = key.endswith("one_block")
        rb = fetch[name]["FETCH_SIZE"] * 1024 * read_scale
        wb = write[name]["WRITE_SIZE"] * 1024 * write_scale
        k = {"read_bytes": rb, "write_bytes": wb}
        for c, short in SQ_KEYS.items():
            if c in sq.get(name, {}):
                k[short] = sq[name][c]
        rec["kernels"][key] = k
        a = alg / 2 if one else alg
        print(f"{name:58s} {fetch[name]['FETCH_SIZE']:10.1f} {write[name]['WRITE_SIZE']:10.1f} "
              f"{rb / 2**20:9.1f} {wb / 2**20:9.1f} {(rb + wb) / a:9.3f}")
    if sq:
        print()
        print(f"{'kernel':58s} {'waves':>8s} {'VALU':>11s} {'VALU/wave':>9s} {'LDS':>9s} {'LDSconfl':>9s} "
              f"{'WAIT_LDS':>10s}")
        for key, name in COUNTER_KERNELS.items():
            q = sq.get(name)
            if not q or "SQ_WAVES" not in q:
                continue
            print(f"{name:58s} {q['SQ_WAVES']:8.0f} {q.get('SQ_INSTS_VALU', 0):11.0f} "
                  f"{q.get('SQ_INSTS_VALU', 0) / q['SQ_WAVES']:9.1f} {q.get('SQ_INSTS_LDS', 0):9.0f} "
                  f"{q.get('SQ_LDS_BANK_CONFLICT', 0):9.0f} {q.get('SQ_WAIT_INST_LDS', 0):10.0f}")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {TRAFFIC_FILE}")


def copy_rate(torch, wl, n=50):
    """torch's plain device copy of one 2048^2 FP32 state (128 MiB read and
    128 MiB written): average microseconds, GB/s and bytes moved per copy."""
    src = torch.empty((wl.grid.ny, wl.grid.nx, 4), dtype=torch.complex64, device="cuda")
    src.real.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(n):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / n
    nbytes = 2 * src.numel() * src.element_size()
    del src, dst
    return us, nbytes / (us * 1e-6) / 1e9, nbytes


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_precision(qw, wl, prec, steps, warmup, torch, sim=None):
    sim = sim or qw.Sim(wl.grid, prec, beam=wl.beam)
    if warmup:
        sim.init_packet(wl.packet)
        sim.step(warmup, 0.0, wl.dt)
    sim.init_packet(wl.packet)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps, 0.0, wl.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    obs = sim.observables(wl.obs)
    return sim, elapsed, obs


def kernel_times(qw, sim, wl, steps, torch):
    sim.init_packet(wl.packet)
    torch.cuda.synchronize()
    qw.qw_kernel_timing(sim.ctx, True)
    sim.step(steps, 0.0, wl.dt)
    cnt_r, ms_r, cnt_c, ms_c = qw.qw_kernel_times(sim.ctx, sim.stream())
    qw.qw_kernel_timing(sim.ctx, False)
    return {"row": (cnt_r, ms_r), "col": (cnt_c, ms_c)}


def batch_section(qw, W, torch, steps, single_steps):
    """Batching workload: 96 seeded instances of 256^2 / 512^2 / 1024^2 FP32.

    Autotunes the batch, times `steps` batched steps (one launch per pass over
    all instances, graph-captured step loop), then the per-pass kernel times,
    then the same instances advanced one by one with the single-instance call
    for `single_steps` steps each.  Per-step work is the same in every step, so
    the two rates compare directly.
    """
    wls = W.batch_instances(seed=0)
    cells = sum(w.grid.nx * w.grid.ny for w in wls)
    log(f"batch: {len(wls)} instances, {cells} cells; autotune")
    bt = qw.Batch([(w.grid, w.beam) for w in wls], qw.QW_F32)
    bt.init_packets([w.packet for w in wls])
    rows = bt.autotune(W.DT, reps=10)
    chosen = {"row": {}, "col": {}}
    for kind, pass_ in ((0, "row"), (1, "col")):
        best = {}
        for r in rows:
            if int(r[0]) == kind and (int(r[1]) not in best or r[3] < best[int(r[1])][1]):
                best[int(r[1])] = (int(r[2]), r[3])
        for lg, (v, _) in sorted(best.items()):
            chosen[pass_][str(1 << lg)] = bt.schedule(lg, v)
    launches = {}
    for kind, pass_ in ((2, "row"), (3, "col")):
        cand = [(r[3], int(r[1])) for r in rows if int(r[0]) == kind]
        launches[pass_ + "_wg_per_cu"] = min(cand)[1] if cand else 0
    # middle steps: graph replays (0) against the step loop (k workgroups per CU)
    def loop_name(w):
        return "graph" if w == 0 else ("instance" if w == qw.QW_LOOP_INSTANCE else f"loop_{w}")
    middle = {loop_name(int(r[1])): round(r[3], 2) for r in rows if int(r[0]) == 4}
    cand = [(r[3], int(r[1])) for r in rows if int(r[0]) == 4]
    launches["loop_wg_per_cu"] = min(cand)[1] if cand else 0
    bt.init_packets([w.packet for w in wls])
    bt.step(20, 0.0, W.DT)
    bt.init_packets([w.packet for w in wls])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(steps, 0.0, W.DT)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    value = cells * steps / tb
    log(f"batch: {steps} steps in {tb:.3f} s -> {value:.4e} cell-steps/s")
    qw.qw_batch_kernel_timing(bt.b, True)
    bt.step(min(200, steps), 0.0, W.DT)
    cnt_r, ms_r, cnt_c, ms_c = qw.qw_batch_kernel_times(bt.b, bt.stream())
    qw.qw_batch_kernel_timing(bt.b, False)
    bt.close()
    row_us, col_us = 1e3 * ms_r / max(cnt_r, 1), 1e3 * ms_c / max(cnt_c, 1)
    sims = []
    for w in wls:
        sm = qw.Sim(w.grid, qw.QW_F32, beam=w.beam)
        sm.init_packet(w.packet)
        sims.append(sm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sm in sims:
        sm.step(single_steps, 0.0, W.DT)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for sm in sims:
        sm.close()
    single = cells * single_steps / ts
    log(f"batch: one by one {single:.4e} cell-steps/s; speedup {value / single:.3f}")
    return {"workload": "96 instances, N in {256, 512, 1024} (seed 0), w0 ~ U[2,16] lambda, A0 ~ U[0.05,1], "
                        "p0y ~ U[0,0.3] k_L, spin +-1, FP32",
            "instances": len(wls), "cells": cells, "steps": steps, "value": value, "unit": "cell-steps/s",
            "ms_per_step": 1e3 * tb / steps, "GBps": round(128 * value / 1e9, 1),
            "single_value": single, "single_steps": single_steps,
            "speedup_batched_vs_single": value / single,
            "avg_launch_us": {"row": round(row_us, 2), "col": round(col_us, 2)},
            "middle_step_us_autotune": middle,
            "small_batch": loop_small(qw, W, torch),
            "tiny_batch": loop_small(qw, W, torch, n_inst=512, n=64),
            "pass_GBps": {"row": round(64 * cells / (row_us * 1e-6) / 1e9, 1),
                          "col": round(64 * cells / (col_us * 1e-6) / 1e9, 1)},
            "schedules": chosen, "launch": launches}


def loop_small(qw, W, torch, n_inst=8, n=256, steps=641):
    """A launch-bound batch (n_inst instances of n^2 FP32): microseconds per
    step with graph replays, with the grid-wide step loop at every workgroup
    count per CU that fits and with one workgroup per instance, and whether
    the final states agree bit for bit."""
    import numpy as np
    cases = []
    for i in range(n_inst):
        g = W.square_box(n, n // 32)
        cases.append((g, W.BeamSpec(a0=0.3 + 0.1 * (i % 8), w0=2.0 * W.LAMBDA_L, ramp_periods=0.0),
                      W.PacketSpec(sigma_x=1.0)))
    out, ref = {}, None
    fit = 0
    for loop in (0, 1, 2, qw.QW_LOOP_INSTANCE):
        bt = qw.Batch([(g, b) for g, b, _ in cases], qw.QW_F32)
        fit = bt.set_loop(-1)
        if loop > fit:
            bt.close()
            continue
        bt.set_loop(loop)
        bt.init_packets([p for _, _, p in cases])
        bt.step(steps, 0.0, W.DT)
        bt.init_packets([p for _, _, p in cases])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.step(steps, 0.0, W.DT)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t0) / steps
        st = [bt.state(i) for i in range(n_inst)]
        bt.observables([W.obs_for(g, p, spin0=p.spin) for g, _, p in cases])  # raises if a barrier wait failed
        bt.close()
        same = None if ref is None else all(np.array_equal(a, b) for a, b in zip(st, ref))
        ref = st if ref is None else ref
        name = "graph" if loop == 0 else ("instance" if loop == qw.QW_LOOP_INSTANCE else f"loop_{loop}")
        out[name] = {"us_per_step": round(us, 2), "bitwise_equal": same}
    log(f"batch: small batch {n_inst}x{n}^2 {out}")
    return {"workload": f"{n_inst} instances of {n}^2 FP32, {steps} steps", "loop_fits_per_cu": fit, **out}


def learned_section(qw, W, torch, batch=4096, reps=50):
    """Surrogate network (4 nets, 5 -> 4 x 256 GELU -> 6) on the matrix cores:
    one training step (forward, back-propagation, Adam) on a batch of 4096 and
    ensemble predictions of 1 and 4096 queries.  The products of a training
    step total 3 x 2 x (5 + 3 x 256 + 6) x 256 x batch x nets flops (forward,
    input gradient, weight gradient; the first layer's input gradient is not
    formed); the MFMA roofline is the dense BF16 peak."""
    import numpy as np
    s = W.SURROGATE_SHAPE
    shift, scale = W.surrogate_input_map()
    net = qw.MLP(s["n_in"], s["width"], s["depth"], s["n_out"], s["n_nets"], max_batch=batch, shift=shift,
                 scale=scale)
    net.set_params(torch.from_numpy(np.concatenate(
        [W.mlp_init_params(k, s["n_in"], s["width"], s["depth"], s["n_out"]) for k in range(s["n_nets"])])))
    rng = np.random.default_rng(0)
    lo = np.array([r[0] for r in W.SURROGATE_INPUT_RANGES])
    hi = np.array([r[1] for r in W.SURROGATE_INPUT_RANGES])
    x = torch.as_tensor(lo + (hi - lo) * rng.random((batch, 5)), dtype=torch.float32, device="cuda")
    t = torch.as_tensor(rng.standard_normal((batch, 6)), dtype=torch.float32, device="cuda")
    for _ in range(5):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / reps
    w, d = s["width"], s["depth"]
    macs = (s["n_in"] * w + (d - 1) * w * w + w * s["n_out"]) * batch * s["n_nets"]
    flops = 2 * macs * 3 - 2 * s["n_in"] * w * batch * s["n_nets"]
    lat = {}
    for q in (1, batch):
        xq = x[:q].contiguous()
        for _ in range(5):
            net.predict(xq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            m, _ = net.predict(xq)
        torch.cuda.synchronize()
        lat[str(q)] = (time.perf_counter() - t0) / reps
    net.close()
    log(f"learned: train step {step_s * 1e6:.1f} us ({flops / step_s / 1e12:.1f} TFLOP/s); "
        f"predict 1: {lat['1'] * 1e6:.1f} us, {batch}: {lat[str(batch)] * 1e6:.1f} us")
    return {"train_step_us": step_s * 1e6, "batch": batch, "nets": s["n_nets"], "train_step_flops": flops,
            "roofline": {"bound": "mfma", "achieved": round(flops / step_s / 1e12, 2), "peak": 2500.0,
                         "unit": "TFLOP/s", "frac": flops / step_s / 1e12 / 2500.0,
                         "note": "23 launches of small products per step; the kernels' own durations add up to "
                                 "the step time (measured with rocprofv3), so the step is bound by the products' "
                                 "operand loads and epilogue stores, not by launch gaps"},
            "predict_us": {k: v * 1e6 for k, v in lat.items()}}


def unfused_section(qw, wl, torch, steps=100):
    """The same Strang step written with torch.fft (rocFFT) and torch elementwise ops.

    A timing comparison for the fused kernels, not part of the library: per
    step fft2 -> K(dt) -> ifft2 -> V(t, dt) on the (ny, nx, 4) complex64
    state, with the time-independent K coefficients precomputed (in FP64,
    stored FP32) and V recomputed per step from the paraxial standing wave.
    Also times the bare transforms (fft2 + ifft2, no pointwise work): the
    floor of any design built on a library FFT.  The result after 20 steps
    is checked against the library (relative L2 of the state).
    """
    g, b = wl.grid, wl.beam
    dev = torch.device("cuda")
    nx, ny, c, dt = g.nx, g.ny, g.c, wl.dt
    f64 = torch.float64
    x = g.x_min + (g.lx / nx) * torch.arange(nx, dtype=f64, device=dev)
    y = g.y_min + (g.ly / ny) * torch.arange(ny, dtype=f64, device=dev)
    kl = 2.0 * math.pi / b.lambda_l
    omega = c * kl
    t_ramp = b.ramp_periods * b.lambda_l / c
    env = torch.exp(-(y / b.w0) ** 2)[:, None]
    ay0 = (b.a0 * env * torch.cos(kl * x)[None, :]).float()
    ax0 = (b.a0 * env * (2.0 * y / (kl * b.w0 ** 2))[:, None] * torch.sin(kl * x)[None, :]).float()
    if not b.longitudinal:
        ax0.zero_()
    px = (2.0 * math.pi / g.lx) * torch.fft.fftfreq(nx, d=1.0 / nx, dtype=f64, device=dev)[None, :]
    py = (2.0 * math.pi / g.ly) * torch.fft.fftfreq(ny, d=1.0 / ny, dtype=f64, device=dev)[:, None]
    en = c * torch.sqrt(c * c + px * px + py * py)
    kc = torch.cos(en * dt).float()
    ks = (torch.sin(en * dt) / en).float()
    pm = (c * torch.complex(px.expand(ny, nx), -py.expand(ny, nx))).to(torch.complex64)
    pp = pm.conj()
    cc = float(c * c)

    def s_of(t):
        f = math.sin(math.pi * t / (2.0 * t_ramp)) ** 2 if t < t_ramp else 1.0
        return f * math.cos(omega * t)

    def v_apply(psi, t, tau):
        s = s_of(t)
        ax, ay = s * ax0, s * ay0
        am = torch.sqrt(ax * ax + ay * ay)
        th = (c * tau) * am
        cth = torch.cos(th)
        sn = torch.where(am > 0, torch.sin(th) / torch.where(am > 0, am, torch.ones_like(am)),
                         torch.full_like(am, c * tau))
        m = torch.complex(ax, -ay)
        p1, p2, p3, p4 = psi.unbind(-1)
        ms = -1j * sn * m
        msc = -1j * sn * m.conj()
        return torch.stack((cth * p1 + ms * p4, cth * p2 + msc * p3, cth * p3 + ms * p2, cth * p4 + msc * p1), -1)

    def k_apply(phi):
        p1, p2, p3, p4 = phi.unbind(-1)
        h = torch.stack((cc * p1 + pm * p4, cc * p2 + pp * p3, -cc * p3 + pm * p2, -cc * p4 + pp * p1), -1)
        return kc[..., None] * phi - 1j * ks[..., None] * h

    def body(psi, k):
        phi = torch.fft.fft2(psi, dim=(0, 1))
        psi = torch.fft.ifft2(k_apply(phi), dim=(0, 1))
        return v_apply(psi, (k + 1) * dt, dt)

    def run(psi, n):
        psi = v_apply(psi, 0.0, 0.5 * dt)
        for k in range(n):
            phi = torch.fft.fft2(psi, dim=(0, 1))
            psi = torch.fft.ifft2(k_apply(phi), dim=(0, 1))
            psi = v_apply(psi, (k + 1) * dt, dt if k < n - 1 else 0.5 * dt)
        return psi

    sim = qw.Sim(g, qw.QW_F32, beam=b)
    sim.init_packet(wl.packet)
    psi0 = sim.psi.clone()
    n_chk = 20
    sim.step(n_chk, 0.0, dt)
    ref = run(psi0, n_chk)
    torch.cuda.synchronize()
    rel = float(torch.linalg.vector_norm(ref - sim.psi) / torch.linalg.vector_norm(sim.psi))
    sim.close()

    psi = psi0.clone()
    for k in range(5):
        psi = body(psi, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        psi = body(psi, k)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / steps
    for _ in range(3):
        psi = torch.fft.ifft2(torch.fft.fft2(psi, dim=(0, 1)), dim=(0, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        psi = torch.fft.ifft2(torch.fft.fft2(psi, dim=(0, 1)), dim=(0, 1))
    torch.cuda.synchronize()
    fft_s = (time.perf_counter() - t0) / steps
    log(f"unfused (torch.fft + elementwise): {step_s * 1e3:.3f} ms/step, bare fft2+ifft2 {fft_s * 1e3:.3f} ms; "
        f"state vs library after {n_chk} steps: rel L2 {rel:.2e}")
    return {"ms_per_step": step_s * 1e3, "fft_only_ms_per_step": fft_s * 1e3,
            "rel_l2_vs_library_20_steps": rel, "steps_timed": steps,
            "note": "torch.fft (rocFFT) + torch elementwise ops, same step; comparison only"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50_000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--timing-steps", type=int, default=2000)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--batch-steps", type=int, default=2000,
                    help="steps of the batching workload (96 instances) to time; 0 skips it")
    ap.add_argument("--batch-single-steps", type=int, default=500,
                    help="steps per instance when the same instances run one by one")
    ap.add_argument("--no-learned", action="store_true", help="skip the surrogate network timing")
    ap.add_argument("--no-unfused", action="store_true",
                    help="skip the torch.fft (rocFFT) comparison of the same step")
    ap.add_argument("--precision", choices=("f32", "f64"), default="f32",
                    help="arithmetic of the timed propagation (f64 skips the FP64 comparison leg)")
    ap.add_argument("--record-counters", metavar="DIR",
                    help="write the traffic record from rocprofv3 --pmc runs under DIR (fetch/, write/, sq/, "
                         "copy_fetch/, copy_write/) and exit; runs without a GPU")
    ap.add_argument("--small-batch", action="store_true",
                    help="only run the launch-bound batches (8 instances of 256^2, 512 of 64^2, FP32) with "
                         "graph replays and with the step loops, and print that comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time torch's plain device copy of one 2048^2 FP32 state (128 MiB read + "
                         "128 MiB written), the reference for bandwidth and traffic counters")
    a = ap.parse_args()
    if a.record_counters:
        record_counters(a.record_counters)
        return
    key = a.precision
    label = key.upper().replace("F", "FP")
    if key == "f64":
        a.no_f64 = True  # the timed run is the FP64 one
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the 2048^2 propagation is "
              "measured on a single GPU, with no sharding across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2307_01571_amd import qw
    from paper_2307_01571_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    qw.lib()
    wl = W.large()
    cells = wl.grid.nx * wl.grid.ny

    if a.small_batch:
        print(json.dumps({"small_batch": loop_small(qw, W, torch),
                          "tiny_batch": loop_small(qw, W, torch, n_inst=512, n=64)}), flush=True)
        return

    if a.copy_probe:
        us, gbs, nbytes = copy_rate(torch, wl)
        print(json.dumps({"probe": "torch copy", "bytes_read": nbytes // 2, "bytes_written": nbytes // 2,
                          "avg_us": us, "GBps": gbs}), flush=True)
        return

    # Untimed, before the timed region: the per-launch durations of the two
    # passes (HIP events around every launch, for the roofline) over
    # --timing-steps steps, and the plain copy of the state.  Both also bring
    # the GPU to its working clocks, so a short timed region measures the
    # same steady state as a long one.
    prec = qw.QW_F32 if key == "f32" else qw.QW_F64
    sim32 = qw.Sim(wl.grid, prec, beam=wl.beam)
    kt = kernel_times(qw, sim32, wl, a.timing_steps, torch)
    copy_us, copy_gbs, _ = copy_rate(torch, wl)

    log(f"{label} {wl.grid.nx}x{wl.grid.ny}: warmup {a.warmup}, timed {a.steps} steps")
    sim32, t32, obs32 = run_precision(qw, wl, prec, a.steps, a.warmup, torch, sim=sim32)
    value = cells * a.steps / t32
    log(f"{label}: {t32:.3f} s, {value:.4e} cell-steps/s, {1e3 * t32 / a.steps:.4f} ms/step")

    per = {}
    for k, (cnt, ms) in kt.items():
        avg_s = ms / max(cnt, 1) / 1e3
        gbs = BYTES_PER_CELL_PASS[key] * cells / avg_s / 1e9
        per[k] = {"launches": int(cnt), "avg_us": avg_s * 1e6, "GBps": gbs}
        log(f"  {k} pass: {cnt:.0f} launches, avg {avg_s * 1e6:.2f} us, {gbs:.0f} GB/s algorithmic")
    dom = max(per, key=lambda k: per[k]["avg_us"])
    dom_name = "col_pass" if dom == "col" else "row_pass"
    counters = measured_counters(dom_name) if key == "f32" else None  # the traffic record is of the FP32 passes
    traffic = None if counters is None else counters["bytes"]
    roofline = {"bound": "hbm", "kernel": dom_name,
                "achieved": round(per[dom]["GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(per[dom]["GBps"] / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / (per[dom]["avg_us"] * 1e-6) / 1e9, 1),
                "traffic_bytes_per_launch": traffic,
                "bytes_per_launch": BYTES_PER_CELL_PASS[key] * cells,
                "avg_launch_us": {k: round(v["avg_us"], 3) for k, v in per.items()},
                # the timed region as a whole: the two passes' algorithmic
                # bytes per step over the measured step time.  There the
                # middle passes of the two Dirac blocks run as two concurrent
                # chains of per-block launches, so one kernel's tail overlaps
                # the other chain's work; the per-launch figures above are of
                # whole-state launches, one at a time on one stream.
                "step_GBps": round(2 * BYTES_PER_CELL_PASS[key] * cells * a.steps / t32 / 1e9, 1)}
    roofline["step_frac"] = round(roofline["step_GBps"] / HBM_PEAK_GBS, 4)
    if counters is not None and counters["valu_insts"]:
        # the second limit: wave-level FP32 VALU issue (no packed FP32), one
        # instruction per SIMD every 4 cycles: 256 CUs x 4 SIMDs x 2.4 GHz / 4
        rate = counters["valu_insts"] / (per[dom]["avg_us"] * 1e-6) / 1e9
        roofline["valu"] = {"insts_per_launch": counters["valu_insts"], "achieved": round(rate, 1),
                            "peak": VALU_PEAK_GINST, "unit": "G wave-instructions/s",
                            "frac": round(rate / VALU_PEAK_GINST, 4)}
    sim32.close()
    # the same traffic as one pass, moved by a plain copy (timed above): the attainable HBM rate
    roofline["copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(per[dom]["GBps"] / copy_gbs, 4)
    log(f"plain copy of the state: {copy_us:.2f} us, {copy_gbs:.0f} GB/s; {dom} pass at "
        f"{roofline['frac_of_copy']:.3f} of it")

    extra = {}
    if not a.no_f64:
        log(f"FP64 reference run, {a.steps} steps")
        sim64, t64, obs64 = run_precision(qw, wl, qw.QW_F64, a.steps, 0, torch)
        sim64.close()
        o32 = qw.unpack_observables(obs32, wl.obs.n_max)
        o64 = qw.unpack_observables(obs64, wl.obs.n_max)
        err = {}
        for key in ("P", "Pp", "Pm"):
            err[key] = float(np.max(np.abs(np.array(o32[key]) - np.array(o64[key]))))
        err["P_flip"] = abs(o32["P_flip"] - o64["P_flip"])
        err["P_neg"] = abs(o32["P_neg"] - o64["P_neg"])
        err["norm_drift_f32"] = o32["norm"] - 1.0
        err["max_abs_prob"] = max(err["P"], err["Pp"], err["Pm"], err["P_flip"])
        # relative errors only of values above the FP32 floor (about 1e-9):
        # a run too short to diffract has P_+1 and P_flip at rounding level
        n_max = wl.obs.n_max
        p1, flip = o64["P"][n_max + 1], o64["P_flip"]
        if p1 > 1e-9:
            err["P_plus1_rel"] = abs(o32["P"][n_max + 1] - p1) / p1
        if flip > 1e-9:
            err["P_flip_rel"] = err["P_flip"] / flip
        if p1 <= 1e-9 or flip <= 1e-9:
            err["note"] = (f"after {a.steps} steps P_+1 = {p1:.2e} and P_flip = {flip:.2e} (FP64) are at rounding "
                           "level: no relative errors; the 5e4-step default run diffracts")
        extra["f64"] = {"value": cells * a.steps / t64, "ms_per_step": 1e3 * t64 / a.steps,
                        "speedup_f32_over_f64": t64 / t32}
        extra["accuracy_vs_f64"] = err
        extra["probabilities_f64"] = {"P": o64["P"], "Pp": o64["Pp"], "Pm": o64["Pm"],
                                      "P_flip": o64["P_flip"], "P_neg": o64["P_neg"]}
        log(f"FP64: {t64:.3f} s; FP32 max |dP| = {err['max_abs_prob']:.3e}")

    def section(name, fn):
        # the context sections must not cost the headline line: a failure is
        # logged and recorded in place of the section's figures
        try:
            extra[name] = fn()
        except Exception as e:  # noqa: BLE001
            log(f"{name} section failed: {e!r}")
            extra[name] = {"error": repr(e)}

    def unfused():
        u = unfused_section(qw, wl, torch)
        u["fused_ms_per_step"] = 1e3 * t32 / a.steps
        u["speedup_fused_over_unfused"] = u["ms_per_step"] / u["fused_ms_per_step"]
        u["speedup_fused_over_fft_only"] = u["fft_only_ms_per_step"] / u["fused_ms_per_step"]
        return u

    if a.batch_steps > 0:
        section("batch", lambda: batch_section(qw, W, torch, a.batch_steps, a.batch_single_steps))
    if not a.no_learned:
        section("learned", lambda: learned_section(qw, W, torch))
    if not a.no_unfused:
        section("unfused_rocfft", unfused)

    # oracle on a bounded sample: the same grid and field, a few steps
    import oracle
    G = oracle.Grid(wl.grid.nx, wl.grid.ny, wl.grid.x_min, wl.grid.y_min, wl.grid.lx, wl.grid.ly, wl.grid.c)
    b = wl.beam
    B = oracle.Beam(b.mode, b.a0, b.lambda_l, b.w0, b.ramp_periods, b.longitudinal, b.ux, b.uy)
    p = wl.packet
    P = oracle.Packet(p.p0x, p.p0y, p.x0, p.y0, p.sigma_x, p.spin)
    psi = oracle.init_packet(G, P)
    tc = time.perf_counter()
    psi = oracle.step_n(G, B, psi, 1, 0.0, wl.dt)
    one = time.perf_counter() - tc
    n_cpu = max(1, min(200, int(a.cpu_budget / max(one, 1e-6))))
    tc = time.perf_counter()
    oracle.step_n(G, B, psi, n_cpu, wl.dt, wl.dt)
    cpu_s = time.perf_counter() - tc
    cpu_value = cells * n_cpu / cpu_s
    n_threads = oracle.get_threads()
    log(f"oracle: {n_cpu} steps in {cpu_s:.1f} s on {n_threads} threads -> {cpu_value:.3e} cell-steps/s")
    # the same on one host thread: one step (the oracle's sums do not depend on the thread count)
    oracle.set_threads(1)
    tc = time.perf_counter()
    oracle.step_n(G, B, psi, 1, wl.dt, wl.dt)
    cpu1_s = time.perf_counter() - tc
    oracle.set_threads(n_threads)
    cpu1_value = cells / cpu1_s
    log(f"oracle: 1 step in {cpu1_s:.1f} s on 1 thread -> {cpu1_value:.3e} cell-steps/s")
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass

    out = {
        "metric": "spinor-cell steps/s at 2048^2 FP32 vs FP64 @1e-4 prob error; %HBM roofline",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * t32 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": key,
        "data": "synthetic",
        "config": {"workload": f"grid2048_box64_w16_a0.5 Strang steps (Dirac split-operator, {label}, "
                               "FP64 phases and reductions)",
                   "nx": wl.grid.nx, "ny": wl.grid.ny, "box_wavelengths": 64, "w0_wavelengths": 16,
                   "a0": wl.beam.a0, "dt": wl.dt, "steps": a.steps},
        "roofline": roofline,
        "cpu_baseline": {"value": cpu_value, "unit": "cell-steps/s", "cores": n_threads,
                         "kind": "oracle",
                         "sample": f"{n_cpu} FP64 steps of the same 2048x2048 workload after 1 step",
                         "one_thread_value": cpu1_value, "cpu_model": cpu_model},
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
