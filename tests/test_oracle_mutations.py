"""Planted mistakes in the oracle must fail the pins.

Each case copies oracle/tplbm_oracle.c into a temporary directory, plants
one plausible mistake by a textual edit (the edit must match the source the
stated number of times, so a case cannot silently stop applying), builds the
copy with the oracle's own flags, routes the oracle binding through it, and
requires every pin named in the case to fail.  The committed oracle passes
all of these pins (tests/test_oracle_pins.py, tests/test_oracle_lattice.py).

A second test shows why the D1Q3 and D3Q19 equilibria divide by the weight's
denominator (r / 18) instead of multiplying by a rounded weight (w * r): the
rounded constant biases every node's mass the same way, and a periodic box
drifts linearly."""
import contextlib
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from tests import oracle_pins as P
from tests import test_oracle_lattice as L

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "tplbm_oracle.c")


def _build_variant(tmp, name, edits):
    src = open(SRC).read()
    for old, new, count in edits:
        assert src.count(old) == count, (name, old, src.count(old))
        src = src.replace(old, new)
    path = os.path.join(tmp, f"{name}.c")
    with open(path, "w") as fh:
        fh.write(src)
    so = os.path.join(tmp, f"lib{name}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-fopenmp", "-o", so, path, "-lm"])
    return so


@contextlib.contextmanager
def _routed_through(orc, so):
    saved = orc._lib
    orc._lib = orc.load_build(so)
    try:
        yield
    finally:
        orc._lib = saved


def _pins(orc, crit):
    """Name -> zero-argument callable running one pin."""
    pins = {}
    for c in P.TRANSPORT_CASES:
        pins[f"transport-{c[0]}-{c[3]}-{len(c[1])}d"] = lambda c=c: P.pin_transport(orc, c)
    for c in P.WORK_CASES:
        pins[f"work-{c[0]}"] = lambda c=c: P.pin_adiabatic_work(orc, crit, c)
    for form in (1, 2):
        for o in ("xz", "yz"):
            pins[f"slab-{form}-{o}"] = (lambda form=form, o=o:
                                        P.pin_d3q19_slab_equals_d2q9(orc, crit, form, o))
    pins["rates"] = lambda: P.pin_relaxation_rate_mapping(orc, crit)
    pins["sound"] = lambda: P.pin_sound_wave_decay(orc)
    pins["mrt-bgk"] = lambda: L.test_tau_one_mrt_li_equals_bgk_guo_plus_isotropic_sigma_term(
        orc, crit)
    pins["momentum-balance-2"] = lambda: L.test_periodic_box_conserves_mass_and_balances_momentum(
        orc, crit, 2)
    pins["collision-momentum"] = lambda: L.test_collision_conserves_mass_and_adds_the_force_to_momentum(
        orc, (1.0, 0.7, 1.3, 0.9, 1.1, 0.8))
    pins["shear-axis"] = lambda: L.test_shear_wave_decays_at_the_mrt_viscosity(orc, 0.8, "axis")
    pins["shear-diagonal"] = lambda: L.test_shear_wave_decays_at_the_mrt_viscosity(
        orc, 0.8, "diagonal")
    pins["cross-lattice-1"] = lambda: L.test_cross_lattice_equivalence_on_x_uniform_columns(
        orc, crit, 1)
    return pins


# name, edits (old, new, expected count), pins that must fail
MUTATIONS = [
    ("advection-sign", [
        ("double adv = -(w->ux[n] * gx + w->uy[n] * gy);",
         "double adv = (w->ux[n] * gx + w->uy[n] * gy);", 1),
        ("return -w->u[y] * gy + P->kappa", "return w->u[y] * gy + P->kappa", 1),
        ("return -(w->ux[n] * gx + w->uy[n] * gy + w->uz[n] * gz) + P->kappa",
         "return (w->ux[n] * gx + w->uy[n] * gy + w->uz[n] * gz) + P->kappa", 1)],
     ["transport-D1Q3-axis-1d", "transport-D2Q9-axis-2d", "transport-D2Q9-diagonal-2d",
      "transport-D3Q19-axis-3d"]),
    ("work-term-without-1/rho", [
        ("/ (rho * P->cv) * orc_eos_dpdT", "/ (P->cv) * orc_eos_dpdT", 3)],
     ["work-D1Q3", "work-D2Q9", "work-D3Q19"]),
    ("work-term-sign", [
        ("double work = -Tf[n] / (rho * P->cv)", "double work = Tf[n] / (rho * P->cv)", 1)],
     ["work-D2Q9"]),
    ("conduction-without-1/rho", [
        ("P->kappa / (rho * P->cv)", "P->kappa / (P->cv)", 3)],
     ["transport-D1Q3-axis-1d", "transport-D2Q9-axis-2d", "transport-D3Q19-axis-3d"]),
    ("heun-to-forward-euler", [
        ("T[n] + 0.5 * (w->k1[n] + k2)", "T[n] + w->k1[n] + 0.0 * k2", 2),
        ("T[y] + 0.5 * (w->k1[y] + k2)", "T[y] + w->k1[y] + 0.0 * k2", 1)],
     ["transport-D1Q3-axis-1d", "transport-D2Q9-diagonal-2d", "transport-D3Q19-axis-3d"]),
    ("d3q19-shan-chen-weights-1/3-1/24", [
        ("(c2 == 1) ? 1.0 / 6.0 : 1.0 / 12.0", "(c2 == 1) ? 1.0 / 3.0 : 1.0 / 24.0", 1)],
     ["slab-1-xz", "slab-2-yz"]),
    ("d3q19-zou-he-without-transverse-terms", [
        ("] - Nx;", "];", 1), ("] + Nx;", "];", 1), ("] - Ny;", "];", 1), ("] + Ny;", "];", 1)],
     ["slab-1-xz", "slab-1-yz"]),
    ("d3q19-zou-he-without-the-y-terms", [
        ("] - Ny;", "];", 1), ("] + Ny;", "];", 1)],
     ["slab-1-yz", "slab-2-yz"]),
    ("tau-e-and-tau-varsigma-swapped", [
        ("L[1] = 1.0 / P->tau[1];\n    L[2] = 1.0 / P->tau[2];",
         "L[1] = 1.0 / P->tau[2];\n    L[2] = 1.0 / P->tau[1];", 1)],
     ["rates", "sound"]),
    ("tau-nu-takes-tau-q", [
        ("L[7] = 1.0 / P->tau[5];", "L[7] = 1.0 / P->tau[4];", 1)],
     ["rates", "shear-diagonal"]),
    ("gravity-form-2-sign-of-the-mean", [
        ("return -(rho - mean) * P->g;", "return -(rho + mean) * P->g;", 1)],
     ["momentum-balance-2"]),
    ("velocity-with-the-whole-force", [
        ("w->ux[n] = (jx + w->Fx[n] / 2.0) / w->rho[n];",
         "w->ux[n] = (jx + w->Fx[n]) / w->rho[n];", 2),
        ("w->uy[n] = (jy + w->Fy[n] / 2.0) / w->rho[n];",
         "w->uy[n] = (jy + w->Fy[n]) / w->rho[n];", 2)],
     ["mrt-bgk", "collision-momentum"]),
    ("d2q9-moments-with-transposed-M", [
        ("m[k] += M2[k][i] * fl[i]; me[k] += M2[k][i] * fe[i];",
         "m[k] += M2[i][k] * fl[i]; me[k] += M2[i][k] * fe[i];", 1)],
     ["mrt-bgk"]),
    ("d2q9-shan-chen-diagonal-weight-1/6", [
        ("if (c2 == 2) return 1.0 / 12.0;", "if (c2 == 2) return 1.0 / 6.0;", 1)],
     ["mrt-bgk", "slab-1-xz"]),
    ("d3q19-guo-term-without-the-half", [
        ("double guo = 0.5 * W3[i]", "double guo = 1.0 * W3[i]", 1)],
     ["slab-1-xz", "slab-2-yz"]),
    ("d1q3-sigma-term-over-3", [
        ("P->sigma * Xp / 6.0", "P->sigma * Xp / 3.0", 1)],
     ["cross-lattice-1"]),
]


@pytest.mark.parametrize("name,edits,must_fail", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_its_pins(orc, crit, tmp_path, name, edits, must_fail):
    so = _build_variant(str(tmp_path), name.replace("/", "_"), edits)
    pins = _pins(orc, crit)
    survived = []
    with _routed_through(orc, so):
        for pin in must_fail:
            try:
                with np.errstate(all="ignore"):
                    pins[pin]()
            except (AssertionError, RuntimeError, FloatingPointError):
                continue
            survived.append(pin)
    assert not survived, f"{name}: passed {survived}"


def _box_mass_drift(orc, crit, lattice, steps):
    _, T_c, _ = crit
    if lattice == "D1Q3":
        P_ = orc.make_params("D1Q3", ny=64, walls=False, g=0.0)
        shape = (64,)
    else:
        P_ = orc.make_params("D3Q19", nx=4, ny=4, nz=24, walls=False, g=0.0)
        shape = (24, 4, 4)
    rv, rl, _ = orc.coexistence(P_, 0.8 * T_c)
    rho0 = W.layered_density(shape, shape[0] // 2, rl, rv, 1e-2, seed=3)
    f = orc.init_rest(P_, rho0.ravel())
    T = np.full(rho0.size, 0.8 * T_c)
    m0 = f.sum()
    orc.step(P_, f, T, steps)
    return (f.sum() - m0) / m0


@pytest.mark.parametrize("lattice,steps,edit", [
    ("D1Q3", 20000, ("w->fs[y] = 2.0 * r / 3.0 * (1.0", "w->fs[y] = 2.0 / 3.0 * r * (1.0")),
    ("D3Q19", 4000, ("double feq = r / W3DEN[i] * (1.0", "double feq = W3[i] * r * (1.0")),
])
def test_rounded_weight_constants_make_a_periodic_box_drift(orc, crit, tmp_path, lattice, steps,
                                                            edit):
    """Fully periodic, g = 0: mass is conserved exactly in exact arithmetic.
    Dividing by the weight's denominator rounds every population once from
    its exact value (errors of either sign: a random walk, measured
    |drift| ~ 5e-15); multiplying by a rounded weight biases all of them the
    same way (measured -3e-17 and -5e-17 per step).  Over 1e5 steps the
    latter would pass the 1e-12 parity bar."""
    committed = _box_mass_drift(orc, crit, lattice, steps)
    so = _build_variant(str(tmp_path), f"rounded_{lattice}", [(edit[0], edit[1], 1)])
    with _routed_through(orc, so):
        rounded = _box_mass_drift(orc, crit, lattice, steps)
    assert abs(committed) < 2e-14, committed
    assert abs(rounded) > 5e-14 and abs(rounded) > 10 * abs(committed), (rounded, committed)
