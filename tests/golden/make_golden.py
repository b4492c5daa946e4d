"""Write the stored oracle results used by the GPU parity tests.

Every value written here comes from the oracle (``oracle/``) and nothing
else: the seeded workloads are propagated on the CPU in FP64 and the final
observables plus a seeded sample of final cells are stored as JSON text.

    python tests/golden/make_golden.py [name ...] [--threads N]

Names: mid_w2, mid_w4, mid_w8 (512 x 512, 1e4 steps; about 10 minutes each on
8 cores), large_prefix0 (2048 x 2048, first 100 steps), large_prefix_field
(2048 x 2048, 50 steps starting after the switch-on ramp).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2307_01571_amd import workloads as W  # noqa: E402
from helpers import o_grid, o_beam, o_packet, o_obs  # noqa: E402

N_RANDOM_CELLS = 192
N_PEAK_CELLS = 64


def sample_cells(psi: np.ndarray, seed: int):
    """Seeded uniform cells plus the cells of largest density (unique, sorted)."""
    ny, nx, _ = psi.shape
    rng = np.random.default_rng(seed)
    flat = rng.choice(ny * nx, size=N_RANDOM_CELLS, replace=False)
    dens = np.sum(np.abs(psi) ** 2, axis=2).ravel()
    peak = np.argsort(dens)[-N_PEAK_CELLS:]
    idx = np.unique(np.concatenate([flat, peak]))
    return [(int(i // nx), int(i % nx)) for i in idx]


def run(wl: W.Workload, steps: int, t0: float):
    G = o_grid(wl.grid)
    psi0 = oracle.init_packet(G, o_packet(wl.packet))
    t = time.time()
    psi = oracle.step_n(G, o_beam(wl.beam), psi0, steps, t0, wl.dt)
    elapsed = time.time() - t
    obs = oracle.observables(G, psi, o_obs(wl.obs))
    cells = sample_cells(psi, seed=1234)
    vals = [psi[iy, ix] for iy, ix in cells]
    return {
        "workload": wl.to_dict(),
        "steps": steps,
        "t0": t0,
        "observables": [float(v) for v in obs],
        "cells": cells,
        "psi_re": [[float(z.real) for z in v] for v in vals],
        "psi_im": [[float(z.imag) for z in v] for v in vals],
        "oracle_seconds": elapsed,
        "oracle_threads": oracle.get_threads(),
        "generator": "tests/golden/make_golden.py (oracle only)",
    }


def jobs():
    mids = {f"mid_w{int(round(wl.beam.w0 / W.LAMBDA_L))}": wl for wl in W.mid_instances(seed=0)}
    out = {name: (wl, wl.steps, 0.0) for name, wl in mids.items()}
    big = W.large()
    out["large_prefix0"] = (big, 100, 0.0)
    out["large_prefix_field"] = (big, 50, 25 * W.T_L)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads:
        oracle.set_threads(a.threads)
    todo = jobs()
    for name in (a.names or list(todo)):
        wl, steps, t0 = todo[name]
        print(f"[golden] {name}: {wl.grid.nx}x{wl.grid.ny} steps={steps} t0={t0}", flush=True)
        rec = run(wl, steps, t0)
        path = os.path.join(HERE, f"{name}.json")
        with open(path + ".tmp", "w") as f:
            json.dump(rec, f, indent=0)
        os.replace(path + ".tmp", path)
        print(f"[golden] {name}: done in {rec['oracle_seconds']:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    main()
