"""(g, Delta T) configuration diagrams (Sec. VI A; the boiling limits of
Sec. V B lie on them).

For each gravity form, each grid point (g, Delta T / T_c) at the paper's
T_med = 0.75 T_c, h = 100 (101 nodes) and <rho> = 1.3344 rho_c, and each
configuration (L-V, V-L, V-L-V):
  * the sharp-interface theory (tplbm_theory_solve) says whether the
    configuration can exist;
  * the batched lattice (tplbm_batch_*), started in that configuration -- the
    theory's profile where one exists, else a sharp profile with the
    zero-gravity lever rule, its interfaces optionally softened to a tanh --
    and run to rest or a step budget, says whether the configuration
    survives (no unphysical-state flag and the same morphology at the end).
The paper finds its lattice stability limits by walking (g, Delta T) from a
stable point in 0.5% steps; here every point starts directly in the
configuration, so a configuration the lattice can hold only as a metastable
state reached gradually may be reported lost.

Run as ``python -m paper_2301_12869_amd.diagram --out DIR``.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import Batch, eos_coexistence, eos_critical, theory_solve

CONFIGS = ("L-V", "V-L", "V-L-V")
H = 101
T_MED = 0.75
MEAN_REDUCED = 1.3344


def morphology(rho: np.ndarray) -> str:
    """Phases from the bottom up, split at the midpoint between the extreme
    densities ('L-V', 'V-L', 'V-L-V', ...); a profile whose extremes differ by
    less than a factor 2 is one phase ('single')."""
    lo, hi = float(rho.min()), float(rho.max())
    if not np.isfinite(lo) or hi < 2.0 * lo:
        return "single"
    liquid = rho > 0.5 * (lo + hi)
    seq = [liquid[0]]
    for v in liquid[1:]:
        if v != seq[-1]:
            seq.append(v)
    return "-".join("L" if v else "V" for v in seq)


def sharp_start(config: str, H: int, mean: float, rv: float, rl: float):
    """Sharp profile of a configuration with the zero-gravity lever rule:
    liquid length H (mean - rv) / (rl - rv), at the bottom (L-V), the top
    (V-L) or the middle (V-L-V).  Returns (rho, interface heights)."""
    ell = H * (mean - rv) / (rl - rv)
    y = np.arange(H) + 0.5
    if config == "L-V":
        liquid, faces = y < ell, [ell - 0.5]
    elif config == "V-L":
        liquid, faces = y > H - ell, [H - ell - 0.5]
    else:
        liquid, faces = np.abs(y - 0.5 * H) < 0.5 * ell, [0.5 * (H - ell) - 0.5, 0.5 * (H + ell) - 0.5]
    return np.where(liquid, rl, rv), faces


def soften(rho: np.ndarray, interfaces, width: float) -> np.ndarray:
    """Replace each sharp interface by a tanh of the given width (nodes):
    within 4 widths of the interface the density runs from the value just
    outside the band on one side to the value on the other.  width <= 0
    leaves the profile sharp."""
    if width <= 0:
        return rho
    out = rho.copy()
    y = np.arange(rho.size)
    band = 4.0 * width
    for h in interfaces:
        lo, hi = int(np.floor(h - band)), int(np.ceil(h + band))
        if lo < 0 or hi >= rho.size:
            continue  # too close to a wall to soften
        a, b = rho[lo], rho[hi]
        k = np.arange(lo + 1, hi)
        out[k] = a + (b - a) * 0.5 * (1.0 + np.tanh((y[k] - h) / width))
    return out


# start interfaces softened to a tanh 2 nodes wide, and kappa = 0.008 (the
# paper lowers kappa to this value where the method needs it for stability;
# the equilibrium's temperature is linear whatever kappa): with sharp starts
# or kappa = 0.02 the first transient breaks many columns that the theory
# says exist (measured form-1 L-V agreement with the theory: 142 of 275
# points sharp at kappa 0.02, 228 at width 2 and kappa 0.02, 271 at width 2
# and kappa 0.008)
WIDTH = 2.0
KAPPA = 0.008


def sweep(forms, g_values, dt_values, steps: int, tol: float = 1e-9, substeps: int = 2,
          check_every: int = 1000, width: float = WIDTH, log=print, **batch_over):
    """Every (form, g, Delta T / T_c, configuration): theory existence and the
    lattice's verdict.  Returns a list of records (dicts)."""
    rho_c, T_c, _ = eos_critical()
    mean = MEAN_REDUCED * rho_c
    rv, rl, _ = eos_coexistence(T_MED * T_c)
    y = np.arange(H)
    cases = [(form, float(g), float(dt), cfg) for form in forms for g in g_values for dt in dt_values
             for cfg in CONFIGS]
    t0 = time.perf_counter()
    th = theory_solve([(H, (T_MED + dt / 2) * T_c, (T_MED - dt / 2) * T_c, g, form, mean, cfg)
                       for form, g, dt, cfg in cases], substeps=substeps)
    t_theory = time.perf_counter() - t0
    log(f"theory: {len(cases)} configurations, {sum(t['rho'] is not None for t in th)} exist, {t_theory:.1f} s")
    rho0, T0 = [], []
    for (form, g, dt, cfg), t in zip(cases, th):
        r, faces = (t["rho"], t["interfaces"]) if t["rho"] is not None else sharp_start(cfg, H, mean, rv, rl)
        r = soften(r, faces, width)
        rho0.append(r + (mean - r.mean()))
        T0.append((T_MED + dt / 2) * T_c + (-dt * T_c) * y / (H - 1))
    batch_over.setdefault("kappa", KAPPA)
    b = Batch([(H, form, g) for form, g, dt, cfg in cases], **batch_over)
    b.set_state(np.concatenate(rho0), np.concatenate(T0))
    b.set_tuning(check_every=check_every)
    t0 = time.perf_counter()
    res = b.run(tol, steps)
    t_lbm = time.perf_counter() - t0
    rho = b.read("rho")
    b.close()
    log(f"lattice: {len(cases)} columns, {steps} step budget, {t_lbm:.1f} s")
    out = []
    for k, ((form, g, dt, cfg), t) in enumerate(zip(cases, th)):
        status = int(res["status"][k])
        final = "diverged" if status == 1 else morphology(rho[k * H:(k + 1) * H])
        out.append(dict(form=form, g=g, dT=dt, config=cfg, theory=t["rho"] is not None,
                        theory_reasons=t["reasons"], lbm_status=["converged", "diverged", "budget"][status],
                        lbm_steps=int(res["steps"][k]), lbm_final=final, lbm_kept=final == cfg))
    return out, dict(theory_seconds=t_theory, lattice_seconds=t_lbm, columns=len(cases),
                     node_steps=float(np.sum(res["steps"])) * H)


def agreement(records) -> dict:
    """Counts of theory / lattice verdicts per form and configuration."""
    out = {}
    for form in sorted({r["form"] for r in records}):
        for cfg in CONFIGS:
            rs = [r for r in records if r["form"] == form and r["config"] == cfg]
            both = sum(r["theory"] and r["lbm_kept"] for r in rs)
            neither = sum(not r["theory"] and not r["lbm_kept"] for r in rs)
            out[f"form{form} {cfg}"] = dict(points=len(rs), agree=both + neither, both_exist=both,
                                             neither=neither,
                                             theory_only=sum(r["theory"] and not r["lbm_kept"] for r in rs),
                                             lattice_only=sum(not r["theory"] and r["lbm_kept"] for r in rs),
                                             lattice_diverged=sum(r["lbm_final"] == "diverged" for r in rs))
    return out


def render(records, form: int) -> str:
    """Text map: rows Delta T / T_c (top = largest), columns g; each cell
    three characters for L-V, V-L, V-L-V: upper case where theory and lattice
    both keep the configuration, lower case where only the theory has it,
    '+' where only the lattice keeps it, '.' where neither, '!' where the
    lattice diverged and the theory has no solution."""
    rs = [r for r in records if r["form"] == form]
    gs = sorted({r["g"] for r in rs})
    dts = sorted({r["dT"] for r in rs}, reverse=True)
    key = {(r["g"], r["dT"], r["config"]): r for r in rs}
    letters = dict(zip(CONFIGS, ("A", "B", "C")))
    lines = [f"form {form}: A = L-V, B = V-L, C = V-L-V; columns g = " + " ".join(f"{g:.1e}" for g in gs)]
    for dt in dts:
        cells = []
        for g in gs:
            c = ""
            for cfg in CONFIGS:
                r = key[(g, dt, cfg)]
                if r["theory"] and r["lbm_kept"]:
                    c += letters[cfg]
                elif r["theory"]:
                    c += letters[cfg].lower()
                elif r["lbm_kept"]:
                    c += "+"
                elif r["lbm_final"] == "diverged":
                    c += "!"
                else:
                    c += "."
            cells.append(c)
        lines.append(f"dT/Tc {dt:+.2f} | " + " ".join(cells))
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--forms", default="1,2")
    ap.add_argument("--g-max", type=float, default=3e-4)
    ap.add_argument("--n-g", type=int, default=13)
    ap.add_argument("--dt-max", type=float, default=0.5)
    ap.add_argument("--n-dt", type=int, default=11)
    ap.add_argument("--steps", type=int, default=1_000_000)
    ap.add_argument("--kappa", type=float, default=KAPPA)
    ap.add_argument("--width", type=float, default=WIDTH, help="tanh width of the start's interfaces (nodes)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    forms = [int(f) for f in args.forms.split(",")]
    gs = np.linspace(-args.g_max, args.g_max, args.n_g)
    dts = np.linspace(-args.dt_max, args.dt_max, args.n_dt)
    recs, info = sweep(forms, gs, dts, args.steps, width=args.width, kappa=args.kappa,
                       log=lambda m: print(m, flush=True))
    summary = dict(info, agreement=agreement(recs), steps=args.steps, kappa=args.kappa, width=args.width)
    json.dump(dict(summary=summary, records=recs), open(os.path.join(args.out, "diagram.json"), "w"), indent=1)
    with open(os.path.join(args.out, "diagram.txt"), "w") as fh:
        for f in forms:
            fh.write(render(recs, f) + "\n\n")
    print(json.dumps(summary, indent=1))
    for f in forms:
        print(render(recs, f))


if __name__ == "__main__":
    main()
