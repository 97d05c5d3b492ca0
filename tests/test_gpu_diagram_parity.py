"""The batched columns against the oracle in the regime of the configuration
diagrams (Sec. VI A): 101-node columns at T_med = 0.75 T_c with linear wall
temperatures (Delta T != 0), kappa = 0.008, <rho> = 1.3344 rho_c, negative
and positive g in both gravity forms, started from V-L and V-L-V profiles
with tanh interfaces two nodes wide (the diagram sweep's starts), run to
max|u| < 1e-9 or 1e5 steps.  Statuses and stopping levels must be the
oracle's, and the end profiles within 1e-12."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
TOL = 1e-12
H, T_MED, MEAN_REDUCED, KAPPA = 101, 0.75, 1.3344, 0.008
CHECK, MAX_STEPS, STEADY = 1000, 100_000, 1e-9

# (gravity form, g, Delta T / T_c, start configuration)
CASES = [
    (1, -2e-5, 0.2, "V-L"),
    (1, -2e-5, 0.2, "V-L-V"),
    (2, -2e-5, 0.1, "V-L"),
    (2, -4e-5, -0.1, "V-L-V"),
    (1, -1e-4, -0.3, "V-L"),
    (2, -1e-4, 0.3, "V-L-V"),
    (1, 3e-5, 0.3, "V-L-V"),
    (2, -6e-5, 0.0, "V-L"),
]


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


def test_diagram_regime_columns_match_the_oracle(T, orc, crit):
    from paper_2301_12869_amd.diagram import morphology, sharp_start, soften

    rho_c, T_c, _ = crit
    mean = MEAN_REDUCED * rho_c
    rv, rl, _ = orc.coexistence(orc.make_params("D1Q3", ny=3), T_MED * T_c)
    y = np.arange(H)
    starts, temps, want = [], [], []
    for form, g, dt, cfg in CASES:
        r, faces = sharp_start(cfg, H, mean, rv, rl)
        r = soften(r, faces, 2.0)
        r = r + (mean - r.mean())
        Tl = (T_MED + dt / 2) * T_c + (-dt * T_c) * y / (H - 1)
        starts.append(r)
        temps.append(Tl)
        P = orc.make_params("D1Q3", ny=H, g=g, gravity_form=form, kappa=KAPPA)
        f = orc.init_rest(P, r)
        TT = Tl.copy()
        n, st = orc.run_to_steady(P, f, TT, STEADY, CHECK, MAX_STEPS)
        m = orc.macro(P, f, TT)
        want.append((n, st, m["rho"], TT))
    b = T.Batch([(H, form, g) for form, g, _, _ in CASES], kappa=KAPPA)
    b.set_state(np.concatenate(starts), np.concatenate(temps))
    b.set_tuning(shape=0, check_every=CHECK)
    res = b.run(STEADY, MAX_STEPS)
    grho, gT = b.read("rho"), b.read("T")
    statuses = []
    for k, ((form, g, dt, cfg), (n, st, orho, oT)) in enumerate(zip(CASES, want)):
        got_st = T.COL_STATUS[res["status"][k]]
        end = morphology(orho) if st != "diverged" else "-"
        _log(f"form {form} g {g:+.0e} dT {dt:+.1f} {cfg}: oracle {st} at {n} ({end}), "
             f"gpu {got_st} at {res['steps'][k]}")
        statuses.append(st)
        assert got_st == st
        if st != "diverged":
            assert res["steps"][k] == n
            assert np.abs(b.column(grho, k) - orho).max() / orho.max() < TOL
            assert np.abs(b.column(gT, k) - oT).max() / oT.max() < TOL
    b.close()
    # the set covers columns that settle, that run out of steps, and that fail
    assert len(set(statuses)) >= 2, statuses
