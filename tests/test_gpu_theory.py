"""The lattice against the sharp-interface theory on the paper's example
(Sec. IV B: h = 100, i.e. 101 nodes, <rho> = 1.3344 rho_c, T_bot = 0.85 T_c,
T_top = 0.65 T_c, g = 2e-5, both gravity forms).

The D2Q9 lattice starts from the theory's profile (shifted to the column's
mass) with the linear temperature and runs 3e5 steps; its steady state is
then compared with the theory.  The paper reports the density in agreement
away from the diffuse interface, the normal pressure close to the theory for
F = rho g and offset by about 5% for F = (rho - <rho>) g.  The bounds below
are those observations with margin (measured: liquid density within 0.13%,
pressure offsets -1.5 .. -2.3% (form 1) and -4.7 .. -5.0% (form 2),
interface within 0.1 node).  An approximate physics check, not a parity test.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

H, NX, STEPS = 101, 4, 300_000


@pytest.fixture(scope="module")
def T():
    import torch

    import paper_2301_12869_amd as T

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    T.load_library()
    return T


def _interface(r):
    mid = 0.5 * (r.max() + r.min())
    k = int(np.nonzero(r < mid)[0][0])
    return k - 1 + (r[k - 1] - mid) / (r[k - 1] - r[k])


@pytest.mark.parametrize("form", [1, 2])
def test_lattice_steady_state_matches_the_theory(T, form):
    rho_c, T_c, _ = T.eos_critical()
    mean, Tb, Tt, g = 1.3344 * rho_c, 0.85 * T_c, 0.65 * T_c, 2e-5
    (th,) = T.theory_solve([(H, Tb, Tt, g, form, mean, "L-V")], substeps=8)
    h = th["interfaces"][0]
    y = np.arange(H)
    rho0 = th["rho"] + (mean - th["rho"].mean())
    T0 = Tb + (Tt - Tb) * y / (H - 1)
    print(f"form {form}: theory interface {h:.3f}, {STEPS} steps on {NX}x{H}", flush=True)
    lat = T.Lattice(T.make_params(T.D2Q9, nx=NX, ny=H, walls=True, gravity_form=form, g=g))
    lat.set_state(np.tile(rho0[:, None], (1, NX)), np.tile(T0[:, None], (1, NX)))
    lat.step(STEPS)
    d = lat.diagnostics()
    r = lat.read("rho").reshape(H, NX)
    p = lat.read("p_nn").reshape(H, NX)
    lat.close()
    assert d["flags"] == 0 and d["max_u"] < 3e-6
    assert np.ptp(r, axis=1).max() < 1e-12 * r.max()  # stays x-uniform
    r, p = r[:, 0], p[:, 0]
    liquid = (y >= 3) & (y < h - 6)
    vapour = (y > h + 8) & (y <= H - 4)  # the vapour side of the interface is wider
    er = (r - th["rho"]) / th["rho"]
    ep = (p - th["p"]) / np.abs(th["p"])
    pl, pv = np.median(ep[liquid]), np.median(ep[vapour])
    print(f"  liquid rho {np.abs(er[liquid]).max():.2e}, vapour rho {np.median(er[vapour]):+.2e}, "
          f"p offset liquid {pl:+.3e} vapour {pv:+.3e}, interface {_interface(r):.3f}", flush=True)
    assert np.abs(er[liquid]).max() < 5e-3
    assert np.abs(er[vapour]).max() < 0.12
    assert abs(_interface(r) - h) < 0.5
    if form == 1:
        assert abs(pl) < 0.035 and abs(pv) < 0.035
    else:
        assert -0.07 < pl < -0.035 and -0.07 < pv < -0.035
