"""Learned warm start for the column sweep.

The pipeline, all on the GPU through the library's C ABI:
  1. draw columns of the sweep (heights, gravities, temperatures, forms, mean
     densities) and run them with the batched solver from the plain
     liquid-below-vapour start; the columns that end without a flag and
     nearly at rest give (column, rho(y), T(y)) training profiles;
  2. train the 1-D convolutional network on those profiles (tplbm_net_*:
     BF16 matrix-core forward/backward, Adam on FP32 master weights);
  3. seed held-out columns with the network's profiles (mean density
     renormalised, wall temperatures kept) and let the batched solver run
     them to steady state; the solver decides what the steady state is.

Run as ``python -m paper_2301_12869_amd.warmstart --out DIR`` to generate
data, train and evaluate; the parameters are written to DIR/warmstart_params.npy.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import Batch, Net, eos_coexistence, eos_critical, theory_solve

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "warmstart_params.npy")

# the sweep's draw: heights 128..2048, g log-uniform in [1e-6, 1e-4],
# isothermal T/T_c uniform in [0.6, 0.95], gravity form 1 or 2, mean density
# uniform between the coexistence densities, 1e-3 relative density noise
NOISE = 1e-3


class Columns:
    """A draw of columns: (height, form, g) for the solver, T/T_c and
    <rho>/rho_c for the network, and the plain liquid-below-vapour start."""

    def __init__(self, n: int, seed: int, h_min: int = 128, h_max: int = 2048):
        import workloads as W

        self.rho_c, self.T_c, _ = eos_critical()
        d = W.column_draws(n, seed, h_min=h_min, h_max=h_max)
        self.n = n
        self.height = d["height"].astype(np.int64)
        self.form = d["form"].astype(np.int64)
        self.g = d["g"]
        self.t_reduced = d["t_reduced"]
        rho, T, rvl = [], [], []
        for k in range(n):
            H = int(self.height[k])
            Tk = self.t_reduced[k] * self.T_c
            rv, rl, _ = eos_coexistence(Tk)
            rvl.append((rv, rl))
            rho.append(W.column_initial_density(H, rv + d["fill"][k] * (rl - rv), rl, rv, NOISE,
                                                int(d["seed"][k])))
            T.append(np.full(H, Tk))
        self.rho0 = np.concatenate(rho)
        self.T0 = np.concatenate(T)
        self.offsets = np.concatenate([[0], np.cumsum(self.height)])
        # the exact mean of each start: the mass the steady state must carry
        mean = np.add.reduceat(self.rho0, self.offsets[:-1]) / self.height
        self.mean_reduced = mean / self.rho_c
        # where a flat interface would sit without gravity (lever rule)
        rvl = np.array(rvl)
        self.lever_height = self.height * (mean - rvl[:, 0]) / (rvl[:, 1] - rvl[:, 0])

    def solver_columns(self, idx=None):
        idx = range(self.n) if idx is None else idx
        return [(int(self.height[k]), int(self.form[k]), float(self.g[k])) for k in idx]

    def net_columns(self, idx=None):
        idx = range(self.n) if idx is None else idx
        return [(int(self.height[k]), int(self.form[k]), float(self.t_reduced[k]), float(self.g[k]),
                 float(self.mean_reduced[k]), float(self.lever_height[k])) for k in idx]

    def take(self, arr, idx):
        return np.concatenate([arr[self.offsets[k]:self.offsets[k + 1]] for k in idx])


CHANNELS = (8, 64, 64, 64, 64, 64, 2)
TAPS = 5


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in), fan_in = 5 C_in) drawn from
    the seeded SplitMix64 stream, zero biases; the parameter layout of
    tplbm_net_set_params."""
    import workloads as W

    parts, k = [], 0
    for l in range(len(CHANNELS) - 1):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        n = cout * TAPS * cin
        parts.append(np.sqrt(6.0 / (TAPS * cin)) * W.uniform_pm1(seed, n, start=k))
        k += n
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def generate(cols: Columns, steps: int, tol: float, keep_u: float, chunk: int = 4096, log=print):
    """Run every column from its plain start for at most `steps` steps (or
    until max |u| < tol); keep those that end without a flag and with
    max |u| < keep_u.  Returns (indices, rho, T) of the kept columns."""
    keep, rho, T = [], [], []
    for c0 in range(0, cols.n, chunk):
        idx = list(range(c0, min(cols.n, c0 + chunk)))
        b = Batch(cols.solver_columns(idx))
        b.set_state(cols.take(cols.rho0, idx), cols.take(cols.T0, idx))
        b.set_tuning(shape=2, check_every=100)
        t0 = time.perf_counter()
        res = b.run(tol, steps)
        r, t = b.read("rho"), b.read("T")
        ok = (res["status"] != 1) & (res["max_u"] < keep_u)
        for j in np.nonzero(ok)[0]:
            keep.append(idx[j])
            rho.append(b.column(r, j))
            T.append(b.column(t, j))
        b.close()
        log(f"generate: columns {c0}..{idx[-1]}: {ok.sum()} kept, {(res['status'] == 1).sum()} diverged, "
            f"{time.perf_counter() - t0:.1f} s")
    return np.array(keep, dtype=np.int64), rho, T


def train(net: Net, n_data: int, heights, epochs: int, batch_nodes: int, lr0: float, lr1: float,
          seed: int, log=print, val=None):
    """Adam with a cosine learning-rate schedule from lr0 to lr1 over
    minibatches of whole columns (about batch_nodes nodes each, in a seeded
    shuffled order).  val: optional callable returning a validation loss."""
    rng = np.random.default_rng(seed)
    batches_per_epoch = max(1, int(np.ceil(heights.sum() / batch_nodes)))
    total = epochs * batches_per_epoch
    step, hist = 0, []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(n_data)
        cur, nodes, losses = [], 0, []
        for k in order:
            cur.append(int(k))
            nodes += int(heights[k])
            if nodes >= batch_nodes or len(cur) == net.config.max_cols:
                lr = lr1 + 0.5 * (lr0 - lr1) * (1 + np.cos(np.pi * min(step, total) / total))
                losses.append(net.train_step(cur, lr))
                step += 1
                cur, nodes = [], 0
        if cur:
            losses.append(net.train_step(cur, lr1))
            step += 1
        v = val() if val else None
        hist.append(dict(epoch=ep, loss=float(np.mean(losses)), val=v, seconds=time.perf_counter() - t0))
        log(f"train: epoch {ep} loss {np.mean(losses):.3e}" + (f" val {v:.3e}" if v is not None else "")
            + f" ({time.perf_counter() - t0:.1f} s)")
    return hist


def theory_start(cols: Columns, substeps: int = 1):
    """Sharp-interface L-V equilibria of the columns (tplbm_theory_solve on
    host threads) as a start: node densities shifted to the column's exact
    mass, the column's uniform temperature.  Columns without an L-V solution
    keep the plain start.  Returns (rho, T, mask of the columns without one)."""
    tc = [(int(cols.height[k]), cols.t_reduced[k] * cols.T_c, cols.t_reduced[k] * cols.T_c,
           float(cols.g[k]), int(cols.form[k]), float(cols.mean_reduced[k] * cols.rho_c), "L-V")
          for k in range(cols.n)]
    sol = theory_solve(tc, substeps=substeps)
    rho = cols.rho0.copy()
    missing = np.zeros(cols.n, dtype=bool)
    for k, s in enumerate(sol):
        a, b = cols.offsets[k], cols.offsets[k + 1]
        if s["rho"] is None:
            missing[k] = True
            continue
        r = s["rho"]
        rho[a:b] = r + (cols.rho0[a:b].mean() - r.mean())
    return rho, cols.T0.copy(), missing


def evaluate(net: Net, cols: Columns, tol: float, max_steps: int, check_every: int = 100, log=print,
             theory: bool = True):
    """Cold (plain start), warm (network density and temperature), warm_rho
    (network density, the column's uniform temperature) and theory
    (sharp-interface equilibrium) starts of the same columns, each run to
    max |u| < tol or max_steps; returns per-column results and the final
    profiles."""
    out = {}
    sc = cols.solver_columns()
    t0 = time.perf_counter()
    rho_w, T_w = net.predict(cols.net_columns())
    t_pred = time.perf_counter() - t0
    starts = [("cold", (cols.rho0, cols.T0)), ("warm", (rho_w, T_w)), ("warm_rho", (rho_w, cols.T0))]
    if theory:
        t0 = time.perf_counter()
        rho_t, T_t, missing = theory_start(cols)
        out["theory_seconds"] = time.perf_counter() - t0
        out["theory_without_solution"] = missing
        log(f"theory start: {cols.n - missing.sum()} L-V solutions, {missing.sum()} without, "
            f"{out['theory_seconds']:.1f} s")
        starts.append(("theory", (rho_t, T_t)))
    for name, (r, t) in starts:
        b = Batch(sc)
        b.set_state(r, t)
        b.set_tuning(shape=2, check_every=check_every)
        t0 = time.perf_counter()
        res = b.run(tol, max_steps)
        dt = time.perf_counter() - t0
        out[name] = dict(res, seconds=dt, rho=b.read("rho"), T=b.read("T"))
        b.close()
        s = res["status"]
        log(f"evaluate {name}: {(s == 0).sum()} converged, {(s == 1).sum()} diverged, "
            f"{(s == 2).sum()} at the step budget, {dt:.1f} s")
    out["predict_seconds"] = t_pred
    out["rho_pred"], out["T_pred"] = rho_w, T_w
    return out


def main():
    import torch

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--train-cols", type=int, default=44000)
    ap.add_argument("--train-seed", type=int, default=1001)
    ap.add_argument("--gen-steps", type=int, default=1_000_000)
    ap.add_argument("--keep-u", type=float, default=1e-4)
    ap.add_argument("--max-profiles", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch-nodes", type=int, default=32768)
    ap.add_argument("--lr0", type=float, default=2e-3)
    ap.add_argument("--lr1", type=float, default=2e-5)
    ap.add_argument("--eval-cols", type=int, default=1024)
    ap.add_argument("--eval-seed", type=int, default=2002)
    ap.add_argument("--eval-steps", type=int, default=4_000_000)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)

    def log(m):
        print(m, flush=True)

    tr = Columns(args.train_cols, args.train_seed)
    keep, rho, T = generate(tr, args.gen_steps, 1e-9, args.keep_u, log=log)
    keep, rho, T = keep[:args.max_profiles], rho[:args.max_profiles], T[:args.max_profiles]
    log(f"dataset: {len(keep)} profiles, {sum(len(r) for r in rho)} nodes")
    ncol = tr.net_columns(keep)
    nv = max(1, len(keep) // 20)  # last 5% held out for validation
    heights = np.array([c[0] for c in ncol])
    net = Net(tr.rho_c, tr.T_c, max_cols=1024, max_nodes=max(args.batch_nodes + 2048, 2048 * 1024),
              dataset_cols=len(keep), dataset_nodes=int(heights.sum()))
    net.set_params(init_params(7))
    net.set_dataset(ncol, np.concatenate(rho), np.concatenate(T))
    ntr = len(keep) - nv
    vidx = np.arange(ntr, len(keep))

    def val():
        ls, ns = [], []
        for s in range(0, nv, 256):
            j = vidx[s:s + 256]
            ls.append(net.loss_grad(j)[0])
            ns.append(heights[j].sum())
        return float(np.dot(ls, ns) / np.sum(ns))

    torch.cuda.synchronize()
    hist = train(net, ntr, heights[:ntr], args.epochs, args.batch_nodes, args.lr0, args.lr1, 5, log=log,
                 val=val)
    theta = net.get_params()
    np.save(os.path.join(args.out, "warmstart_params.npy"), theta)

    ev = Columns(args.eval_cols, args.eval_seed)
    res = evaluate(net, ev, 1e-9, args.eval_steps, log=log)
    summary = summarize(ev, res)
    summary.update(train_history=hist, dataset_profiles=int(len(keep)), gen_steps=args.gen_steps,
                   keep_u=args.keep_u)
    json.dump(summary, open(os.path.join(args.out, "warmstart_summary.json"), "w"), indent=1)
    log(json.dumps({k: v for k, v in summary.items() if k != "train_history"}))


def summarize(cols: Columns, res: dict) -> dict:
    """Counts, steps and steady-states per hour of cold and warm starts, and
    the agreement of the steady states both reach."""
    c = res["cold"]
    m0 = np.add.reduceat(cols.rho0, cols.offsets[:-1])  # mass of the plain start (= the seeded mass)
    out = {}
    names = [n for n in ("cold", "warm", "warm_rho", "theory") if n in res]
    setup = dict(cold=0.0, warm=res["predict_seconds"], warm_rho=res["predict_seconds"],
                 theory=res.get("theory_seconds", 0.0))
    for name in names:
        r = res[name]
        conv = r["status"] == 0
        secs = r["seconds"] + setup[name]
        out[name] = dict(converged=int(conv.sum()), diverged=int((r["status"] == 1).sum()),
                         budget=int((r["status"] == 2).sum()), seconds=secs,
                         steady_states_per_hour=float(conv.sum() / secs * 3600.0),
                         median_steps_converged=float(np.median(r["steps"][conv])) if conv.any() else None)
    # the prediction against the solver's end state from the plain start
    ok = c["status"] != 1
    pe = []
    for k in np.nonzero(ok)[0]:
        a = c["rho"][cols.offsets[k]:cols.offsets[k + 1]]
        p = res["rho_pred"][cols.offsets[k]:cols.offsets[k + 1]]
        pe.append(float(np.linalg.norm(p - a) / np.linalg.norm(a)))
    if pe:
        out["prediction_rel_l2_median"] = float(np.median(pe))
        out["prediction_rel_l2_q90"] = float(np.quantile(pe, 0.9))
    for name in names[1:]:
        w = res[name]
        both = (c["status"] == 0) & (w["status"] == 0)
        cmp = dict(both_converged=int(both.sum()))
        if both.any():
            same, diffs, dmass, pairs = 0, [], [], []
            for k in np.nonzero(both)[0]:
                a = c["rho"][cols.offsets[k]:cols.offsets[k + 1]]
                b = w["rho"][cols.offsets[k]:cols.offsets[k + 1]]
                pa, pb = interface_positions(a), interface_positions(b)
                rec = dict(column=int(k), height=int(cols.height[k]), morphology_cold=morphology(a),
                           morphology_warm=morphology(b), mass_diff=float(b.sum() - a.sum()),
                           rho_max_rel_diff=float(np.abs(a - b).max() / a.max()))
                if rec["morphology_cold"] == rec["morphology_warm"] and len(pa) == len(pb):
                    same += 1
                    diffs.append(rec["rho_max_rel_diff"])
                    dmass.append(float(abs(b.sum() - a.sum()) / a.sum()))
                    # a flat interface moves by the mass difference over the
                    # density jump; half a node covers where a node straddles it
                    jump = float(a.max() - a.min())
                    shift = float(np.max(np.abs(np.array(pb) - np.array(pa)))) if pa else 0.0
                    rec.update(interface_shift=shift, shift_bound=abs(rec["mass_diff"]) / jump + 0.5)
                pairs.append(rec)
            cmp.update(steps_ratio_median=float(np.median(w["steps"][both] / c["steps"][both])),
                       same_morphology=same)
            if diffs:
                cmp.update(final_rho_max_rel_diff_median=float(np.median(diffs)),
                           final_rho_max_rel_diff_max=float(np.max(diffs)),
                           final_mass_rel_diff_median=float(np.median(dmass)))
            # pairs that settled in different configurations (several steady
            # states of one column can coexist), and same-configuration pairs
            # whose interfaces moved further than their mass difference explains
            other = [p for p in pairs if p["morphology_cold"] != p["morphology_warm"]]
            bad = [p for p in pairs if "interface_shift" in p and p["interface_shift"] > p["shift_bound"]]
            worst = max(pairs, key=lambda p: p["rho_max_rel_diff"])
            cmp.update(shift_within_bound=sum(1 for p in pairs if "interface_shift" in p
                                              and p["interface_shift"] <= p["shift_bound"]),
                       other_configuration=other, violations=bad, largest_difference=worst)
        out[name + "_vs_cold"] = cmp
    # mass the walls add or remove during the transient (the seeded mass is
    # the column's <rho> H for every start)
    if "theory" in res:
        # columns with no L-V equilibrium in theory: what the solver did
        # with them from the plain start
        miss = res["theory_without_solution"]
        out["theory"]["without_solution"] = int(miss.sum())
        out["theory"]["without_solution_cold_status"] = {
            v: int((c["status"][miss] == k).sum()) for k, v in ((0, "converged"), (1, "diverged"), (2, "budget"))}
        out["theory"]["with_solution_cold_status"] = {
            v: int((c["status"][~miss] == k).sum()) for k, v in ((0, "converged"), (1, "diverged"), (2, "budget"))}
    for name in names:
        r = res[name]
        conv = r["status"] == 0
        if conv.any():
            out[name]["mass_drift_rel_median"] = float(np.median(np.abs(r["mass"][conv] - m0[conv]) / m0[conv]))
    return out


def morphology(rho: np.ndarray) -> str:
    """Phase sequence from the bottom ('L-V', 'V-L', 'V-L-V', ...), split at
    the midpoint between the extreme densities."""
    from .diagram import morphology as phases

    return phases(rho)


def interface_positions(rho: np.ndarray) -> list:
    """Heights (in nodes from node 0) where a profile crosses the midpoint
    between its extreme densities, by linear interpolation between nodes."""
    mid = 0.5 * (rho.max() + rho.min())
    d = rho - mid
    out = []
    for k in np.nonzero(np.sign(d[1:]) != np.sign(d[:-1]))[0]:
        out.append(float(k + d[k] / (d[k] - d[k + 1])))
    return out


def interfaces(rho: np.ndarray) -> int:
    """Number of liquid-vapour interfaces of a profile: crossings of the
    midpoint between its extreme densities."""
    mid = 0.5 * (rho.max() + rho.min())
    s = np.sign(rho - mid)
    return int(np.count_nonzero(s[1:] != s[:-1]))


if __name__ == "__main__":
    main()
