"""GPU parity of the D3Q19 update against the oracle's independent D3Q19.

Small lattices are compared node by node (FP64 within 1e-12, FP32-deviation
storage within 1e-5 in density).  The 256^3 workload is checked on sampled
sub-boxes: one step moves information at most four nodes (pull, psi, force,
velocity, two temperature stages), so after s steps the interior of a box,
4s nodes away from its x and y faces, depends only on the initial data inside
it; the oracle runs that box with periodic x, y and the interiors must agree."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch

    import paper_2301_12869_amd as T

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    T.load_library()
    return T


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


RHO_V3 = 0.025  # the density gravity form 3 subtracts (about the vapour's at 0.8 T_c)


def _oracle(orc, shape, walls, form, g, rho0, T0, steps):
    nx, ny, nz = shape
    P = orc.make_params("D3Q19", nx=nx, ny=ny, nz=nz, walls=walls, g=g, gravity_form=form, rho_v=RHO_V3)
    f = orc.init_rest(P, rho0.ravel())
    TT = T0.ravel().copy()
    orc.step(P, f, TT, steps)
    return orc.macro(P, f, TT)


def _gpu(T, shape, walls, form, g, rho0, T0, steps, precision=0, state=None, ref_interval=0):
    nx, ny, nz = shape
    p = T.make_params(T.D3Q19, nx=nx, ny=ny, nz=nz, walls=walls, gravity_form=form, g=g,
                      precision=precision, rho_ref=float(rho0.mean()), rho_v=RHO_V3,
                      state=T.STATE_AUTO if state is None else state, ref_interval=ref_interval)
    lat = T.Lattice(p)
    lat.set_state(rho0, T0)
    lat.step(steps)
    out = {k: lat.read(k) for k in ("rho", "ux", "uy", "uz", "T", "p_nn")}
    out["diag"] = lat.diagnostics()
    lat.close()
    return out


def _state(orc, crit, shape, seed, layers):
    _, T_c, _ = crit
    nx, ny, nz = shape
    P = orc.make_params("D3Q19", nx=nx, ny=ny, nz=nz)
    rv, rl, _ = orc.coexistence(P, 0.8 * T_c)
    rho0 = W.layered_density((nz, ny, nx), layers, rl, rv, 2e-2, seed=seed)
    T0 = W.wall_temperature_field((nz, ny, nx), 0.8 * T_c, 0.86 * T_c, 0.79 * T_c)
    return rho0, T0


@pytest.mark.parametrize("shape,walls,form", [((6, 5, 14), True, 1), ((6, 5, 14), True, 2),
                                              ((7, 4, 9), False, 2), ((1, 1, 20), True, 2),
                                              ((5, 6, 13), True, 3), ((70, 9, 11), True, 2),
                                              ((40, 35, 24), True, 2), ((33, 20, 17), False, 2),
                                              ((4, 3, 3), True, 2), ((3, 2, 3), False, 2)])
def test_small_lattices_fp64(T, orc, crit, shape, walls, form):
    """The moment state (rho, j and T carried between steps) against the
    oracle, on tiles wider than the lattice, several 32 x 16 tiles with ragged
    edges, z segments (24 and 17 planes make three and two) with walls and
    periodic in z, and the shallowest lattices (3 planes: one interior plane
    between two walls, or a periodic stack the march wraps around)."""
    _log(f"case d3q19 fp64 moment state {shape} walls={walls} form={form}")
    rho0, T0 = _state(orc, crit, shape, 5, shape[2] // 3)
    want = _oracle(orc, shape, walls, form, 2e-4, rho0, T0, 200)
    got = _gpu(T, shape, walls, form, 2e-4, rho0, T0, 200, state=T.STATE_MOMENTS)
    for k in ("rho", "T"):
        assert _rel(got[k], want[k]) < 1e-12, (k, _rel(got[k], want[k]))
    for k in ("ux", "uy", "uz"):
        assert np.abs(got[k] - want[k]).max() < 1e-13, k
    assert np.abs(got["p_nn"] - want["p_nn"]).max() / (0.5 * want["rho"].max() ** 2) < 1e-12


@pytest.mark.parametrize("shape,walls,form", [((70, 9, 11), True, 2), ((33, 40, 7), False, 1),
                                              ((40, 35, 12), True, 3), ((1, 1, 20), True, 2),
                                              ((6, 5, 14), True, 1), ((65, 3, 9), False, 2)])
def test_population_state_fp64(T, orc, crit, shape, walls, form):
    """The nineteen-population state (the z-marching kernels) against the
    oracle, on lattices with several 32 x 32 tiles, ragged tile edges, tiles
    wider than the lattice, z segments and both boundary kinds."""
    _log(f"case d3q19 fp64 populations {shape} walls={walls} form={form}")
    rho0, T0 = _state(orc, crit, shape, 11, max(1, shape[2] // 3))
    want = _oracle(orc, shape, walls, form, 2e-4, rho0, T0, 200)
    got = _gpu(T, shape, walls, form, 2e-4, rho0, T0, 200, state=T.STATE_POPULATIONS)
    for k in ("rho", "T"):
        assert _rel(got[k], want[k]) < 1e-12, (k, _rel(got[k], want[k]))
    for k in ("ux", "uy", "uz"):
        assert np.abs(got[k] - want[k]).max() < 1e-13, k
    assert np.abs(got["p_nn"] - want["p_nn"]).max() / (0.5 * want["rho"].max() ** 2) < 1e-12
    assert got["diag"]["flags"] == 0


def test_fp32_deviation_several_tiles(T, orc, crit):
    """FP32 deviations on a lattice of several tiles and z segments."""
    shape = (40, 36, 17)
    rho0, T0 = _state(orc, crit, shape, 12, 6)
    want = _oracle(orc, shape, True, 2, 1e-4, rho0, T0, 300)
    got = _gpu(T, shape, True, 2, 1e-4, rho0, T0, 300, precision=1)
    err = _rel(got["rho"], want["rho"])
    _log(f"  fp32dev {shape} rho rel err {err:.3e}")
    assert err < 1e-5
    assert _rel(got["T"], want["T"]) < 1e-5


@pytest.mark.parametrize("shape,walls,form", [((70, 9, 11), True, 2), ((33, 10, 7), False, 1),
                                              ((40, 12, 9), True, 3)])
def test_moment_state_matches_population_state(T, orc, crit, shape, walls, form):
    """The moment state (the FP64 default) carries (rho, j) and T between
    steps; the nineteen-population state evaluates the same post-collision
    populations, so the two agree to rounding (differently grouped sums, the
    rest population closed by mass or by its closed form), on lattices
    spanning several tiles of both kernels with ragged edges."""
    _log(f"case d3q19 moment vs population {shape} walls={walls} form={form}")
    rho0, T0 = _state(orc, crit, shape, 8, shape[2] // 3)
    pop = _gpu(T, shape, walls, form, 2e-4, rho0, T0, 300)
    mom = _gpu(T, shape, walls, form, 2e-4, rho0, T0, 300, state=T.STATE_MOMENTS)
    for k in ("rho", "T"):
        assert _rel(mom[k], pop[k]) < 1e-13, (k, _rel(mom[k], pop[k]))
    for k in ("ux", "uy", "uz"):
        assert np.abs(mom[k] - pop[k]).max() < 1e-14, k
    assert mom["diag"]["mass"] == pytest.approx(pop["diag"]["mass"], rel=1e-13)
    assert mom["diag"]["flags"] == pop["diag"]["flags"] == 0


def test_moment_state_checkpoint_is_bitwise(T, orc, crit):
    shape = (34, 9, 10)
    rho0, T0 = _state(orc, crit, shape, 9, 3)
    p = T.make_params(T.D3Q19, nx=34, ny=9, nz=10, walls=True, gravity_form=2, g=2e-4, state=T.STATE_MOMENTS)
    a = T.Lattice(p)
    a.set_state(rho0, T0)
    a.step(40)
    blob = a.save_state()
    a.step(25)
    want = {k: a.read(k) for k in ("rho", "uz", "T")}
    a.close()
    b = T.Lattice(p)
    b.load_state(blob)
    b.step(25)
    got = {k: b.read(k) for k in ("rho", "uz", "T")}
    b.close()
    for k in want:
        assert np.array_equal(got[k], want[k]), k


@pytest.mark.parametrize("ref_interval", [-1, 0, 40])
def test_small_lattice_fp32_deviation(T, orc, crit, ref_interval):
    """FP32 deviations from one reference (-1) or per-plane references
    re-centred every 256 (default) or 40 steps, against the FP64 oracle."""
    shape = (6, 6, 24)
    rho0, T0 = _state(orc, crit, shape, 6, 8)
    want = _oracle(orc, shape, True, 2, 1e-4, rho0, T0, 500)
    got = _gpu(T, shape, True, 2, 1e-4, rho0, T0, 500, precision=1, ref_interval=ref_interval)
    err = _rel(got["rho"], want["rho"])
    _log(f"  fp32dev ref_interval={ref_interval} rho rel err {err:.3e}")
    assert err < 1e-5
    assert _rel(got["T"], want["T"]) < 1e-5


def test_full_256_cubed_on_sampled_sub_boxes(T, orc, crit):
    """256^3, periodic x and y, walls in z, liquid in the bottom 64 planes,
    bottom plane at T/T_c = 0.9, bulk 0.8, g = 1e-5, both forms, 2 steps."""
    _, T_c, _ = crit
    n, steps, box = 256, 2, 24
    P = orc.make_params("D3Q19", nx=3, ny=3, nz=3)
    rv, rl, _ = orc.coexistence(P, 0.8 * T_c)
    rho0 = W.layered_density((n, n, n), 64, rl, rv, 1e-3, seed=4)
    T0 = W.wall_temperature_field((n, n, n), 0.8 * T_c, 0.9 * T_c, 0.8 * T_c)
    for form, prec in ((1, 1), (2, 0)):
        _log(f"case d3q19 256^3 form={form} precision={prec}")
        got = _gpu(T, (n, n, n), True, form, 1e-5, rho0, T0, steps, precision=prec)
        grho = got["rho"].reshape(n, n, n)
        for (x0, y0) in ((0, 0), (100, 37), (231, 200)):
            xs = [(x0 + i) % n for i in range(box)]
            ys = [(y0 + i) % n for i in range(box)]
            sub_r = rho0[:, ys][:, :, xs].copy()
            sub_T = T0[:, ys][:, :, xs].copy()
            want = _oracle(orc, (box, box, n), True, form, 1e-5, sub_r, sub_T, steps)
            m = 4 * steps
            wr = want["rho"].reshape(n, box, box)[:, m:box - m, m:box - m]
            gr = grho[:, ys][:, :, xs][:, m:box - m, m:box - m]
            tol = 1e-12 if prec == 0 else 1e-5
            if form == 2:
                # <rho> of the box differs from the lattice's through the
                # seeded noise (about 1e-7 relative over 147 456 nodes), so
                # (rho - <rho>) g differs by about g * 1e-8 per step
                tol = max(tol, 1e-10)
            assert np.abs(gr - wr).max() / wr.max() < tol
