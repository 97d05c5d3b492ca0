"""Phase-change protocol runs (Sec. V A): a column is brought to equilibrium
with its top wall warmer than the target, then the top wall is cooled to the
target and the run continues; a new vapour phase at the (hot) bottom wall is
the boiling the paper predicts from the liquid spinodal.

All columns of a scan run together in the batched sweep
(tplbm_batch_run / tplbm_batch_resume); the start is the sharp-interface
equilibrium of the first stage (the lever-rule profile where there is
none), interfaces softened to a tanh.

The paper's case: gravity form 1, g = 1.5e-5, 101 nodes, <rho> = 1.3344 rho_c,
first-stage T_top = 0.6213 T_c, then T_top lowered to the target; its first
case is T_bot = 0.9083 T_c, T_top = 0.5917 T_c (dT/T_c = 0.3166, T_med = 0.75).
For larger dT the paper changes only the top wall's temperature between the
stages but does not say whether T_bot stays at 0.9083 T_c or moves to keep
T_med = 0.75 T_c; both readings are offered (t_bot fixed, or t_bot=None for
T_bot = (0.75 + dT/2) T_c).  Its lattice keeps the liquid at dT/T_c = 0.3381
and boils at 0.3382 (a vapour layer at the bottom wall by t = 252 500 after
the change, the phases inverted by t = 800 000).

Run as ``python -m paper_2301_12869_amd.protocol --out DIR``.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import Batch, eos_coexistence, eos_critical, theory_solve
from .diagram import MEAN_REDUCED, morphology, sharp_start, soften


def boiling_scan(dts, g: float = 1.5e-5, form: int = 1, H: int = 101, t_bot: float = 0.9083,
                 t_top_first: float = 0.6213, first_steps: int = 2_000_000, first_tol: float = 1e-10,
                 second_steps: int = 1_500_000, chunk: int = 50_000, width: float = 2.0,
                 kappa: float = 0.02, log=print):
    """One column per dT / T_c.  Returns per-column records: the first stage's
    outcome, the steps after the change at which the bottom wall was first
    covered by vapour (None if never), and the morphology at the end."""
    rho_c, T_c, _ = eos_critical()
    mean = MEAN_REDUCED * rho_c
    dts = [float(d) for d in dts]
    n = len(dts)
    T_bot = np.array([((0.75 + d / 2) if t_bot is None else t_bot) * T_c for d in dts])
    t_top1 = np.full(n, t_top_first * T_c)
    t_top2 = T_bot - np.array(dts) * T_c
    y = np.arange(H)
    th = theory_solve([(H, T_bot[k], t_top1[k], g, form, mean, "L-V") for k in range(n)], substeps=4)
    rho0, T0 = [], []
    no_theory = 0
    for k, t in enumerate(th):
        if t["rho"] is not None:
            r, faces = t["rho"], t["interfaces"]
        else:
            # no sharp-interface L-V for the first stage: the lever-rule
            # profile at the mean wall temperature
            no_theory += 1
            rv, rl, _ = eos_coexistence(0.5 * (T_bot[k] + t_top1[k]))
            r, faces = sharp_start("L-V", H, mean, rv, rl)
        r = soften(r, faces, width)
        rho0.append(r + (mean - r.mean()))
        T0.append(T_bot[k] + (t_top1[k] - T_bot[k]) * y / (H - 1))
    b = Batch([(H, form, g)] * n, kappa=kappa)
    b.set_state(np.concatenate(rho0), np.concatenate(T0))
    b.set_tuning(check_every=1000)
    t0 = time.perf_counter()
    r1 = b.run(first_tol, first_steps)
    log(f"first stage: {int((r1['status'] == 0).sum())} of {n} at rest, {int((r1['status'] == 1).sum())} "
        f"diverged ({no_theory} started from the lever rule), {time.perf_counter() - t0:.1f} s")
    rho1 = b.read("rho")
    first = [dict(status=["converged", "diverged", "budget"][int(s)], steps=int(st), max_u=float(u),
                  final="diverged" if s == 1 else morphology(b.column(rho1, k)))
             for k, (s, st, u) in enumerate(zip(r1["status"], r1["steps"], r1["max_u"]))]
    layer = [None] * n
    diverged_at = [None] * n
    b.resume(T_top=t_top2)
    done = 0
    t0 = time.perf_counter()
    while done < second_steps:
        k_steps = min(chunk, second_steps - done)
        r = b.run(0.0, k_steps)
        done += k_steps
        rho = b.read("rho")
        for k in range(n):
            if diverged_at[k] is None and r["status"][k] == 1:
                diverged_at[k] = done - k_steps + int(r["steps"][k])
            if layer[k] is None and diverged_at[k] is None and morphology(b.column(rho, k)).startswith("V"):
                layer[k] = done
        b.resume()
    log(f"second stage: {second_steps} steps in chunks of {chunk}, {time.perf_counter() - t0:.1f} s")
    rho = b.read("rho")
    b.close()
    out = []
    for k in range(n):
        out.append(dict(dT=dts[k], T_bot=T_bot[k] / T_c, T_top_first=t_top_first, T_top=t_top2[k] / T_c,
                        first_stage=first[k], vapour_layer_at=layer[k], diverged_at=diverged_at[k],
                        final=("diverged" if diverged_at[k] is not None else morphology(b.column(rho, k)))))
    return out


def threshold(records):
    """(largest dT that kept the liquid at the bottom through both stages,
    smallest dT whose column grew a vapour layer there after the change),
    over the columns whose first stage ended in L-V."""
    ok = [r for r in records if r["first_stage"]["final"] == "L-V"]
    kept = [r["dT"] for r in ok if r["vapour_layer_at"] is None and r["diverged_at"] is None]
    boiled = [r["dT"] for r in ok if r["vapour_layer_at"] is not None]
    return (max(kept) if kept else None), (min(boiled) if boiled else None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--dt-min", type=float, default=0.31)
    ap.add_argument("--dt-max", type=float, default=0.37)
    ap.add_argument("--n", type=int, default=61)
    ap.add_argument("--kappa", type=float, default=0.02)
    ap.add_argument("--second-steps", type=int, default=1_500_000)
    ap.add_argument("--t-bot", type=float, default=0.9083, help="bottom wall T/T_c; <= 0 keeps T_med = 0.75")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    dts = np.linspace(args.dt_min, args.dt_max, args.n)
    recs = boiling_scan(dts, kappa=args.kappa, second_steps=args.second_steps,
                        t_bot=args.t_bot if args.t_bot > 0 else None, log=lambda m: print(m, flush=True))
    lo, hi = threshold(recs)
    summary = dict(kept_up_to=lo, boiled_from=hi, kappa=args.kappa, t_bot=args.t_bot, records=recs)
    json.dump(summary, open(os.path.join(args.out, "protocol.json"), "w"), indent=1)
    for r in recs:
        print(f"dT/Tc {r['dT']:.4f}: first stage {r['first_stage']['status']} at {r['first_stage']['steps']} "
              f"({r['first_stage']['final']}), "
              f"vapour layer at {r['vapour_layer_at']}, diverged at {r['diverged_at']}, final {r['final']}")
    print(f"liquid kept up to dT/Tc = {lo}; vapour layer from dT/Tc = {hi}")


if __name__ == "__main__":
    main()
