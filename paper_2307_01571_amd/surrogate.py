"""Learned form: a surrogate of the split-operator solver, trained on the
solver's own batched runs, with the solver as fallback.

Inputs of a query: (w0, A0, interaction time T, p0y, spin); outputs: the
probabilities P_0, P_+1, P_-1, P_+2, P_-2 and P_flip the solver reports
(qw_observables) for a 512 x 512 FP32 run of those parameters after time T.

* ``generate``: runs of the batching workload's distribution restricted to
  512^2 (seeded draws), advanced together with qw_batch_step_n; the
  observables are taken every ``snap_every`` steps, so every run gives one
  training sample per snapshot (T = snapshot time).
* ``train``: the 4-net ensemble of qw_mlp (BF16 MFMA kernels) on a fixed
  seeded start, Adam on minibatches, cosine learning-rate decay.
* ``evaluate``: held-out runs (never seen in training) -> error of the
  ensemble mean against the solver, the ensemble spread as error estimate,
  the share of queries the fallback would send to the solver.
* ``SurrogateWithFallback``: answers from the network where the error
  estimate is at most ``tol`` and from the solver elsewhere.

The error estimate is the ensemble spread in standardised units: for each
output the standard deviation of the four nets' predictions divided by that
output's standard deviation over the training targets, the largest of the
six.  The outputs span 1e-12 to 1, so a spread in the outputs' own units
would let the small ones (P_+-2, P_flip) through whatever their error
(measured: an absolute 1e-2 sends no in-distribution query to the solver).
The default tolerance, 0.1 of each output's spread of values, sits above
the nets' typical disagreement on held-out runs (0.02 to 0.07) and below
that of the queries they get wrong; it also implies the absolute 1e-2 on
every output whose training spread is below 0.1 (all six here; train()
checks it), so it is the stricter of the two readings.

Torch serves as device memory and for shuffling minibatches; the network's
arithmetic runs in the library's kernels, the solver's in its own.

    python -m paper_2307_01571_amd.surrogate generate --runs 4096 --seed 0 --out data0.npz
    python -m paper_2307_01571_amd.surrogate train --data data0.npz data1.npz --report out.json
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

N_GRID = 512
STEPS = 20_000
SNAP_EVERY = 1000
FALLBACK_TOL = 0.1  # error estimate (standardised units) above which the solver answers
ABS_TOL = 1e-2      # the absolute probability tolerance the standardised one implies


def _log(*a):
    print("[surrogate]", *a, file=sys.stderr, flush=True)


def select_outputs(obs, n_max: int = 2) -> np.ndarray:
    """(P_0, P_+1, P_-1, P_+2, P_-2, P_flip) from one qw_observables vector."""
    nb = 2 * n_max + 1
    P = obs[1:1 + nb]
    return np.array([P[n_max], P[n_max + 1], P[n_max - 1], P[n_max + 2], P[n_max - 2], obs[1 + 3 * nb]])


def run_inputs(wl: W.Workload, t: float) -> np.ndarray:
    return np.array([wl.beam.w0, wl.beam.a0, t, wl.packet.p0y, float(wl.packet.spin)])


def generate(n_runs: int, seed: int, steps: int = STEPS, snap_every: int = SNAP_EVERY, chunk: int = 1024,
             n: int = N_GRID):
    """Solver data: x [n_runs * snaps][5], y [n_runs * snaps][6], run index per sample."""
    wls = W.batch_instances(seed=seed, count=n_runs, sizes=(n,), steps=steps)
    snaps = steps // snap_every
    xs, ys, rid = [], [], []
    for c0 in range(0, n_runs, chunk):
        part = wls[c0:c0 + chunk]
        tc = time.perf_counter()
        bt = qw.Batch([(w.grid, w.beam) for w in part], qw.QW_F32)
        bt.init_packets([w.packet for w in part])
        specs = [w.obs for w in part]
        for s in range(1, snaps + 1):
            bt.step(snap_every, (s - 1) * snap_every * W.DT, W.DT)
            obs = bt.observables(specs)
            t = s * snap_every * W.DT
            for i, w in enumerate(part):
                xs.append(run_inputs(w, t))
                ys.append(select_outputs(obs[i]))
                rid.append(c0 + i)
            _log(f"runs {c0}..{c0 + len(part) - 1}: snapshot {s}/{snaps} (t = {t:.4f})")
        bt.close()
        _log(f"chunk of {len(part)} runs: {time.perf_counter() - tc:.1f} s")
    return np.array(xs), np.array(ys), np.array(rid)


def solve(params, n: int = N_GRID):
    """Solver answers for arbitrary queries (w0, A0, T, p0y, spin): one batched run
    per query, each advanced to its own T (queries are grouped by step count)."""
    params = np.asarray(params, dtype=np.float64)
    out = np.zeros((len(params), 6))
    ksteps = np.rint(params[:, 2] / W.DT).astype(np.int64)
    for k in np.unique(ksteps):
        idx = np.nonzero(ksteps == k)[0]
        inst, packets, specs = [], [], []
        for i in idx:
            g = W.square_box(n, n // 32)
            b = W.BeamSpec(a0=float(params[i, 1]), w0=float(params[i, 0]))
            p = W.PacketSpec(p0y=float(params[i, 3]), spin=int(round(params[i, 4])))
            inst.append((g, b))
            packets.append(p)
            specs.append(W.obs_for(g, p, spin0=p.spin))
        bt = qw.Batch(inst, qw.QW_F32)
        bt.init_packets(packets)
        if k > 0:
            bt.step(int(k), 0.0, W.DT)
        obs = bt.observables(specs)
        bt.close()
        for j, i in enumerate(idx):
            out[i] = select_outputs(obs[j])
    return out


def make_net(max_batch: int = 4096, seed: int = 0):
    import torch
    s = W.SURROGATE_SHAPE
    shift, scale = W.surrogate_input_map()
    net = qw.MLP(s["n_in"], s["width"], s["depth"], s["n_out"], s["n_nets"], max_batch=max_batch, shift=shift,
                 scale=scale)
    p0 = np.concatenate([W.mlp_init_params(seed + k, s["n_in"], s["width"], s["depth"], s["n_out"])
                         for k in range(s["n_nets"])])
    net.set_params(torch.from_numpy(p0))
    return net


def target_map(y):
    """Per-output (mean, standard deviation) of the training targets; the
    network learns the standardised targets and predicts through the map."""
    y = np.asarray(y, dtype=np.float64)
    mu = y.mean(axis=0)
    sd = y.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


def train(x, y, epochs: int = 200, batch: int = 4096, lr: float = 1e-3, lr_end: float = 1e-5, seed: int = 0,
          net=None):
    """Adam on shuffled minibatches of standardised targets; returns the net
    (predicting in the targets' units) and the loss history (per epoch, mean
    over nets, in standardised units)."""
    import torch
    dev = torch.device("cuda")
    mu, sd = target_map(y)
    xd = torch.as_tensor(x, dtype=torch.float32, device=dev)
    yd = torch.as_tensor((np.asarray(y) - mu) / sd, dtype=torch.float32, device=dev)
    n = xd.shape[0]
    batch = min(batch, n)
    net = net or make_net(max_batch=max(batch, 4096), seed=seed)
    net.set_output_map(mu, sd)
    net.set_spread_weights(1.0 / sd)  # the error estimate in standardised units
    if np.any(sd * FALLBACK_TOL > ABS_TOL):
        _log(f"note: an output's spread of values ({sd.max():.3g}) makes the standardised tolerance "
             f"looser than {ABS_TOL} absolute")
    net.target_mean, net.target_std = mu, sd
    g = torch.Generator(device="cpu").manual_seed(seed)
    loss = torch.zeros(W.SURROGATE_SHAPE["n_nets"], device=dev)
    per_epoch = n // batch
    total = epochs * per_epoch
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        acc = torch.zeros_like(loss)
        for b in range(per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb = xd.index_select(0, idx).contiguous()
            yb = yd.index_select(0, idx).contiguous()
            cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * step / max(total - 1, 1)))
            net.train_step(xb, yb, cur, loss)
            acc += loss
            step += 1
        hist.append(float(acc.mean().item()) / per_epoch)
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            _log(f"epoch {ep}: loss {hist[-1]:.3e}")
    return net, hist


def predict(net, x):
    import torch
    x = np.asarray(x, dtype=np.float64)
    chunk = net.shape.max_batch
    means, spreads = [], []
    for i in range(0, len(x), chunk):
        m, s = net.predict(torch.as_tensor(x[i:i + chunk], dtype=torch.float32, device="cuda"))
        means.append(m.double().cpu().numpy())
        spreads.append(s.double().cpu().numpy())
    return np.concatenate(means), np.concatenate(spreads)


class SurrogateWithFallback:
    """Network answers where the error estimate (ensemble spread in
    standardised units) is <= tol, the solver's elsewhere."""

    def __init__(self, net, tol: float = FALLBACK_TOL):
        self.net = net
        self.tol = tol

    def __call__(self, params):
        mean, spread = predict(self.net, params)
        use = spread > self.tol
        out = mean.copy()
        if np.any(use):
            out[use] = solve(np.asarray(params)[use])
        return out, use, spread


def evaluate(net, x, y, tol: float = FALLBACK_TOL) -> dict:
    """Errors of the ensemble mean against the solver: absolute, and in
    standardised units (each output's error over its training standard
    deviation, the units of the error estimate); each output's RMS error
    relative to its spread over the evaluated set and to the RMS error of the
    constant predictor (the training mean): skill = 1 - (rmse /
    rmse_constant)^2; and how the fallback at tol splits the queries."""
    mean, spread = predict(net, x)
    err = np.abs(mean - y)
    sd = getattr(net, "target_std", np.ones(err.shape[1]))
    err_std = err / sd
    worst = err_std.max(axis=1)
    accept = spread <= tol
    rmse = np.sqrt(np.mean((mean - y) ** 2, axis=0))
    mu = getattr(net, "target_mean", np.mean(y, axis=0))
    rmse0 = np.sqrt(np.mean((mu - y) ** 2, axis=0))
    res = {"samples": int(len(x)), "outputs": list(W.SURROGATE_OUTPUTS),
           "rmse": rmse.tolist(), "rmse_over_std": (rmse / np.maximum(np.std(y, axis=0), 1e-300)).tolist(),
           "skill_vs_constant": (1 - (rmse / np.maximum(rmse0, 1e-300)) ** 2).tolist(),
           "mae": err.mean(axis=0).tolist(), "max_abs": err.max(axis=0).tolist(),
           "max_abs_rel_to_output_max": (err.max(axis=0) / np.maximum(np.abs(y).max(axis=0), 1e-300)).tolist(),
           "max_abs_all": float(err.max()), "max_std_all": float(worst.max()),
           "share_within_tol": float(np.mean(worst <= tol)),
           "fallback_share": float(1 - accept.mean()),
           "mean_std_err_accepted": float(worst[accept].mean()) if accept.any() else None,
           "mean_std_err_fallback": float(worst[~accept].mean()) if (~accept).any() else None,
           "max_std_err_accepted": float(worst[accept].max()) if accept.any() else None,
           "accepted_within_tol": float(np.mean(worst[accept] <= tol)) if accept.any() else None,
           "spread_vs_error_corr": float(np.corrcoef(spread, worst)[0, 1]) if len(x) > 2 else None}
    return res


def latency(net, wl_params, reps: int = 20) -> dict:
    """Surrogate query latency (1 and up to 4096 queries) against the solver for one query."""
    import torch
    x1 = torch.as_tensor(np.asarray(wl_params[:1]), dtype=torch.float32, device="cuda")
    nb = min(4096, net.shape.max_batch)
    xb = torch.as_tensor(np.resize(np.asarray(wl_params), (nb, 5)), dtype=torch.float32, device="cuda")
    for _ in range(3):
        net.predict(x1)
        net.predict(xb)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        m, s = net.predict(x1)
        m.cpu()
    one = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):
        m, s = net.predict(xb)
        m.cpu()
    many = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    solve(np.asarray(wl_params[:1]))
    sol = time.perf_counter() - t
    return {"surrogate_1_query_s": one, f"surrogate_{nb}_queries_s": many, "solver_1_query_s": sol,
            "solver_query_steps": int(round(float(np.asarray(wl_params)[0, 2]) / W.DT)),
            "speedup_1_query": sol / one, "queries_per_s_surrogate": nb / many}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--runs", type=int, default=4096)
    g.add_argument("--seed", type=int, default=0)
    g.add_argument("--steps", type=int, default=STEPS)
    g.add_argument("--snap-every", type=int, default=SNAP_EVERY)
    g.add_argument("--chunk", type=int, default=1024)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--holdout-runs", type=int, default=512)
    t.add_argument("--epochs", type=int, default=200)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--report", required=True)
    a = ap.parse_args(argv)
    qw.lib()
    if a.cmd == "generate":
        tg = time.perf_counter()
        x, y, rid = generate(a.runs, a.seed, a.steps, a.snap_every, a.chunk)
        el = time.perf_counter() - tg
        np.savez(a.out, x=x, y=y, run=rid, seed=a.seed, steps=a.steps, snap_every=a.snap_every, seconds=el)
        _log(f"{a.runs} runs, {len(x)} samples in {el:.1f} s -> {a.out}")
        return
    xs, ys, rs, meta = [], [], [], []
    off = 0
    for f in a.data:
        d = np.load(f)
        xs.append(d["x"])
        ys.append(d["y"])
        rs.append(d["run"] + off)
        off += int(d["run"].max()) + 1
        meta.append({"file": f, "seed": int(d["seed"]), "runs": int(d["run"].max()) + 1,
                     "generate_s": float(d["seconds"])})
    x, y, rid = np.concatenate(xs), np.concatenate(ys), np.concatenate(rs)
    n_runs = off
    rng = np.random.default_rng(12345)
    held = set(rng.choice(n_runs, size=min(a.holdout_runs, n_runs // 4), replace=False).tolist())
    test = np.array([r in held for r in rid])
    tt = time.perf_counter()
    net, hist = train(x[~test], y[~test], epochs=a.epochs, lr=a.lr)
    import torch
    torch.cuda.synchronize()
    train_s = time.perf_counter() - tt
    rep = {"data": meta, "runs": n_runs, "train_samples": int((~test).sum()), "heldout_runs": len(held),
           "heldout_samples": int(test.sum()), "epochs": a.epochs, "train_s": train_s,
           "loss_first": hist[0], "loss_last": hist[-1],
           "train_eval": evaluate(net, x[~test][:20000], y[~test][:20000]),
           "heldout_eval": evaluate(net, x[test], y[test]),
           "latency": latency(net, x[test][:16])}
    with open(a.report, "w") as f:
        json.dump(rep, f, indent=1)
    _log(json.dumps(rep["heldout_eval"]))
    _log(json.dumps(rep["latency"]))


if __name__ == "__main__":
    main()
