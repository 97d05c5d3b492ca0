"""The allocation-free column sweep (tplbm_batch_run_noalloc) against the
workspace sweep (tplbm_batch_create / set_state / run) on the same columns:
two calls in a row, the second with fewer and shorter columns than the
first, both bit for bit equal to tplbm_batch_run (the same kernel; columns
are independent, so the processing order does not change them)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch

    import paper_2301_12869_amd as T

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    T.load_library()
    return T


def _columns(orc, crit, n, seed, hmin, hmax):
    _, T_c, _ = crit
    d = W.column_draws(n, seed, h_min=hmin, h_max=hmax)
    P = orc.make_params("D1Q3", ny=3)
    cols, rho, Tc = [], [], []
    for k in range(n):
        H = int(d["height"][k])
        Tk = d["t_reduced"][k] * T_c
        rv, rl, _ = orc.coexistence(P, Tk)
        mean = rv + d["fill"][k] * (rl - rv)
        cols.append((H, int(d["form"][k]), float(d["g"][k])))
        rho.append(W.column_initial_density(H, mean, rl, rv, 1e-3, int(d["seed"][k])))
        Tc.append(np.full(H, Tk))
    return cols, np.concatenate(rho), np.concatenate(Tc)


def _workspace_run(T, cols, rho, Tc, tol, K, max_steps):
    b = T.Batch(cols)
    b.set_state(rho, Tc)
    b.set_tuning(shape=0, check_every=K)
    res = b.run(tol, max_steps)
    out = res, b.read("rho"), b.read("T")
    b.close()
    return out


def _noalloc_run(T, cols, rho, Tc, tol, K, max_steps, alias=False):
    import torch

    dev = torch.device("cuda")
    r0 = torch.from_numpy(rho).to(dev)
    t0 = torch.from_numpy(Tc).to(dev)
    r1 = r0 if alias else torch.empty_like(r0)
    t1 = t0 if alias else torch.empty_like(t0)
    res = torch.empty(32 * len(cols), dtype=torch.uint8, device=dev)
    T.batch_run_noalloc(cols, r0, t0, r1, t1, res, tol, max_steps, K)
    return T.col_results(res), r1.cpu().numpy(), t1.cpu().numpy()


@pytest.mark.parametrize("alias", [False, True])
def test_noalloc_sweep_equals_the_workspace_sweep(T, orc, crit, alias):
    cases = [
        # 40 columns of 100-300 nodes, a fixed budget
        (_columns(orc, crit, 40, seed=23, hmin=100, hmax=300), 1e-8, 100, 3000),
        # then fewer, shorter columns, run to steady state
        (_columns(orc, crit, 12, seed=17, hmin=12, hmax=72), 1e-8, 50, 60000),
    ]
    for (cols, rho, Tc), tol, K, max_steps in cases:
        _log(f"case noalloc alias={alias}: {len(cols)} columns, {rho.size} nodes, budget {max_steps}")
        want, wrho, wT = _workspace_run(T, cols, rho, Tc, tol, K, max_steps)
        got, grho, gT = _noalloc_run(T, cols, rho, Tc, tol, K, max_steps, alias=alias)
        # diverged columns carry NaN in both runs: NaN counts as equal to NaN
        for key in ("steps", "status", "mass", "max_u"):
            assert np.array_equal(got[key], want[key], equal_nan=True), key
        assert np.array_equal(grho, wrho, equal_nan=True)
        assert np.array_equal(gT, wT, equal_nan=True)
        _log(f"  statuses {np.bincount(got['status'], minlength=3)}")


def test_noalloc_rejects_more_columns_than_its_scratch_holds(T):
    import torch

    n = 8193
    cols = [(3, 1, 1e-5)] * n
    x = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    res = torch.empty(32 * n, dtype=torch.uint8, device="cuda")
    with pytest.raises(T.TplbmError, match="ESHAPE"):
        T.batch_run_noalloc(cols, x, x, x, x, res, 1e-9, 10, 10)
