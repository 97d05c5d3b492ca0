"""Write the goldens of the full-size GPU parity tests with the FP64 oracle.

Only ``oracle/`` (and the seeded input generators of ``workloads/``, which
hold none of the method's arithmetic) is called here; every stored value is
the oracle's.  The files are compact: a fixed sample of nodes and per-layer
sums, not whole fields.  The scalars the inputs were built from (coexistence
densities and critical temperature from the oracle's EOS) are stored too, so
that the GPU tests rebuild bit-identical inputs from them.

    python tests/golden/make_full_size.py c2        # 1024x2048 D2Q9, 1000 steps, both forms (~7 min, 8 threads)
    python tests/golden/make_full_size.py c4        # 256^3 D3Q19, 100 steps, both forms (~15 min)
    python tests/golden/make_full_size.py columns   # config-3 columns (seed 3) run to max|u| < 1e-9
    python tests/golden/make_full_size.py all

Workloads (as the benchmark and the paper's parameters set them):
- C2: D2Q9 1024 x 2048, walls at the bottom and top rows, liquid in the
  bottom 64 rows and vapour above (Maxwell densities at 0.8 T_c), bottom wall
  0.9 T_c, top wall and bulk 0.8 T_c, 1e-3 density noise (seed 2), g = 1e-5,
  F = rho g and F = (rho - <rho>) g.
- C4: D3Q19 256^3, periodic x and y, walls in z, liquid in the bottom 64
  planes, bottom plane 0.9 T_c, bulk 0.8 T_c, noise seed 4, g = 1e-5, both
  forms.
- Columns: the 4096-column draw of seed 3 (heights 128..2048, g log-uniform
  in [1e-6, 1e-4], T/T_c in [0.6, 0.95], both forms, liquid below vapour at a
  mean density between the coexistence densities, 1e-3 noise).  Columns are
  tried shortest first (short columns relax fastest) until 64 of them
  converge within the step budget or COL_MAX_TRIED have been tried; every
  tried column's status and stopping level is kept, and the profiles of the
  converged ones.  The file is rewritten after every group of columns, so an
  interrupted run leaves the columns finished so far.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

C2_STEPS, C4_STEPS = 1000, 100
COL_TOL, COL_CHECK, COL_MAX_STEPS, COL_WANT = 1e-9, 100, 2_000_000, 64
# columns tried at most: converging columns thin out with height (55 of the
# 832 shortest converge within the step budget, none of the next 240), so
# the search stops there if 64 have not converged by then
COL_MAX_TRIED = 832

# sampled nodes: rows/planes across the walls, the interface and the bulk
C2_ROWS = [0, 1, 2, 3, 31, 32, 62, 63, 64, 65, 66, 67, 68, 100, 511, 1024, 2000, 2045, 2046, 2047]
C2_COLS = list(range(5, 1024, 16))
C4_PLANES = [0, 1, 2, 62, 63, 64, 65, 66, 128, 254, 255]
C4_XY = [(x, y) for y in range(3, 256, 16) for x in range(11, 256, 16)]


def path(name: str) -> str:
    return os.path.join(HERE, name)


def c2(threads: int):
    rho_c, T_c, _ = oracle.critical()
    P0 = oracle.make_params("D2Q9", nx=3, ny=3)
    rv, rl, _ = oracle.coexistence(P0, 0.8 * T_c)
    nx, ny = 1024, 2048
    rho0 = W.layered_density((ny, nx), 64, rl, rv, 1e-3, seed=2)
    T0 = W.wall_temperature_field((ny, nx), 0.8 * T_c, 0.9 * T_c, 0.8 * T_c)
    oracle.set_threads(threads)
    out = dict(rho_l=rl, rho_v=rv, T_c=T_c, steps=C2_STEPS, rows=np.array(C2_ROWS), cols=np.array(C2_COLS))
    for form in (1, 2):
        t0 = time.time()
        P = oracle.make_params("D2Q9", nx=nx, ny=ny, walls=True, g=1e-5, gravity_form=form)
        f = oracle.init_rest(P, rho0.ravel())
        T = T0.ravel().copy()
        d = oracle.step(P, f, T, C2_STEPS)
        m = oracle.macro(P, f, T)
        sel = np.ix_(C2_ROWS, C2_COLS)
        for k in ("rho", "ux", "uy", "p_nn"):
            out[f"form{form}_{k}"] = m[k].reshape(ny, nx)[sel].copy()
        out[f"form{form}_T"] = T.reshape(ny, nx)[sel].copy()
        out[f"form{form}_row_rho"] = m["rho"].reshape(ny, nx).sum(axis=1)
        out[f"form{form}_row_T"] = T.reshape(ny, nx).sum(axis=1)
        out[f"form{form}_flags"] = d["flags"]
        print(f"c2 form {form}: {time.time() - t0:.0f} s, flags {d['flags']}", flush=True)
    np.savez_compressed(path("c2_d2q9_1024x2048_1000_steps.npz"), **out)


def c4(threads: int):
    rho_c, T_c, _ = oracle.critical()
    P0 = oracle.make_params("D3Q19", nx=3, ny=3, nz=3)
    rv, rl, _ = oracle.coexistence(P0, 0.8 * T_c)
    n = 256
    rho0 = W.layered_density((n, n, n), 64, rl, rv, 1e-3, seed=4)
    T0 = W.wall_temperature_field((n, n, n), 0.8 * T_c, 0.9 * T_c, 0.8 * T_c)
    oracle.set_threads(threads)
    xs = np.array([p[0] for p in C4_XY])
    ys = np.array([p[1] for p in C4_XY])
    out = dict(rho_l=rl, rho_v=rv, T_c=T_c, steps=C4_STEPS, planes=np.array(C4_PLANES), xs=xs, ys=ys)
    for form in (1, 2):
        t0 = time.time()
        P = oracle.make_params("D3Q19", nx=n, ny=n, nz=n, walls=True, g=1e-5, gravity_form=form)
        f = oracle.init_rest(P, rho0.ravel())
        T = T0.ravel().copy()
        d = oracle.step(P, f, T, C4_STEPS)
        m = oracle.macro(P, f, T)
        del f
        for k in ("rho", "ux", "uy", "uz", "p_nn"):
            out[f"form{form}_{k}"] = m[k].reshape(n, n, n)[np.array(C4_PLANES)][:, ys, xs].copy()
        out[f"form{form}_T"] = T.reshape(n, n, n)[np.array(C4_PLANES)][:, ys, xs].copy()
        out[f"form{form}_plane_rho"] = m["rho"].reshape(n, n * n).sum(axis=1)
        out[f"form{form}_plane_T"] = T.reshape(n, n * n).sum(axis=1)
        out[f"form{form}_flags"] = d["flags"]
        del m
        print(f"c4 form {form}: {time.time() - t0:.0f} s, flags {d['flags']}", flush=True)
    np.savez_compressed(path("c4_d3q19_256cubed_100_steps.npz"), **out)


def _column(args):
    H, form, g, T, rho0 = args
    P = oracle.make_params("D1Q3", ny=H, g=g, gravity_form=form)
    f = oracle.init_rest(P, rho0)
    TT = np.full(H, T)
    n, st = oracle.run_to_steady(P, f, TT, COL_TOL, COL_CHECK, COL_MAX_STEPS)
    m = oracle.macro(P, f, TT)
    return n, st, m["rho"], TT


def columns(workers: int):
    rho_c, T_c, _ = oracle.critical()
    d = W.column_draws(4096, 3)
    P0 = oracle.make_params("D1Q3", ny=3)
    order = np.argsort(d["height"], kind="stable")
    conv = 0
    recs = {"height": [], "form": [], "g": [], "T": [], "index": [], "steps": [], "status": [],
            "rho0": [], "rho": [], "Tend": []}
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for start in range(0, len(order), workers):
            chunk = order[start:start + workers]
            args = []
            for k in chunk:
                H = int(d["height"][k])
                Tk = float(d["t_reduced"][k] * T_c)
                rv, rl, _ = oracle.coexistence(P0, Tk)
                mean = rv + d["fill"][k] * (rl - rv)
                r0 = W.column_initial_density(H, mean, rl, rv, 1e-3, int(d["seed"][k]))
                args.append((H, int(d["form"][k]), float(d["g"][k]), Tk, r0))
            for k, a, (n, st, rho, TT) in zip(chunk, args, ex.map(_column, args)):
                if conv >= COL_WANT:
                    break
                recs["height"].append(a[0]); recs["form"].append(a[1]); recs["g"].append(a[2])
                recs["T"].append(a[3]); recs["index"].append(int(k)); recs["steps"].append(n)
                recs["status"].append({"converged": 0, "diverged": 1, "max_steps": 2}[st])
                recs["rho0"].append(a[4])
                recs["rho"].append(rho if st == "converged" else np.full(a[0], np.nan))
                recs["Tend"].append(TT if st == "converged" else np.full(a[0], np.nan))
                conv += st == "converged"
            print(f"columns: {len(recs['index'])} tried, {conv} converged, {time.time() - t0:.0f} s", flush=True)
            _write_columns(recs)
            if conv >= COL_WANT or len(recs["index"]) >= COL_MAX_TRIED:
                break


def _write_columns(recs):
    out = {k: np.array(v) for k, v in recs.items() if k not in ("rho0", "rho", "Tend")}
    for k in ("rho0", "rho", "Tend"):
        out[k] = np.concatenate(recs[k])
    out.update(tol=COL_TOL, check_every=COL_CHECK, max_steps=COL_MAX_STEPS)
    tmp = path("c3_columns_seed3_to_steady.tmp.npz")
    np.savez_compressed(tmp, **out)
    os.replace(tmp, path("c3_columns_seed3_to_steady.npz"))


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    threads = os.cpu_count() or 1
    if what in ("c2", "all"):
        c2(threads)
    if what in ("c4", "all"):
        c4(threads)
    if what in ("columns", "all"):
        columns(threads)
    print(json.dumps({"done": what}))
