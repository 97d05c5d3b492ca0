"""Pins of the oracle's energy update, rate mapping and D3Q19 isotropy.

Each ``pin_*`` function runs the oracle on a small case whose answer the
paper and the mathematics fix independently of the oracle's code, and raises
AssertionError on a mismatch.  They are plain functions (not pytest tests) so
that ``tests/test_oracle_pins.py`` runs them on the oracle as built and
``tests/test_oracle_mutations.py`` runs them on copies of the oracle with a
planted mistake, each of which must fail at least one pin.

What each pin fixes:

- ``pin_transport``: Eq. Energy_Equation linearised about a uniform state of
  an ideal lattice gas (psi = 0 and (dp/dT)_rho = 0, so only advection and
  conduction act) is a constant-coefficient equation.  On a Fourier mode
  exp(i k.x) the isotropic differences of Sec. III have closed-form symbols
  (derived below from the stencil weights), so every Heun step multiplies
  the mode by 1 + lam + lam^2/2 with lam = -i u0.s(k) + kappa l(k)/(rho0 c_v).
  This fixes the sign of the advection term, the 1/(rho c_v) factor of the
  conduction term, and the second-order Runge-Kutta (a forward Euler step has
  no lam^2/2).
- ``pin_adiabatic_work``: with kappa = 0 the same equation and the continuity
  equation (Eq. MassConservation) give, to first order in a small density
  wave at rest, T(t) - T(0) = T0 R Z(eta0) / (rho0 c_v) (rho(t) - rho(0)),
  with (dp/dT)_rho = rho R Z(eta) for the Carnahan-Starling EOS (Eq. EOS).
  This fixes the size and sign of the pressure-work term.  In time, the
  lattice's continuity is second-order accurate about the half level
  n + 1/2 while the energy step holds u at level n, so T^n pairs with the
  density of level n - 1/2, (rho^n + rho^(n-1))/2; compared with rho^n
  itself the relation is off by the phase omega/2 of the sound wave.  What
  is left is the O(k^2) error of the isotropic divergence (sin k against k).
- ``pin_d3q19_slab_equals_d2q9``: D3Q19 on an nx x 1 x nz (or 1 x ny x nz)
  lattice sums, velocity group by velocity group, to D2Q9 on nx x nz: the
  weights 1/3 + 2/18 = 4/9, 1/18 + 2/36 = 1/9, 1/36; the Shan-Chen weights
  1/6 + 2/12 = 1/3 and 1/12 (Eq. ShanChenForce); the isotropic differences;
  half of Guo's forcing term; and the wet-node wall reconstruction with its
  transverse-momentum terms.  The sigma term of Eq. LiFS differs between the
  two in a fourth moment, so the pin runs at sigma = 0.
- ``pin_relaxation_rate_mapping``: Eq. RelaxationMatrix assigns tau_e to the
  moment e, tau_varsigma to varsigma, tau_q to q_x and q_y, tau_nu to p_xx
  and p_xy, and tau_rho and tau_j to conserved moments (no effect).
  Changing one relaxation time must change exactly its own post-collision
  moments, computed with the printed M (Eq. MatrixMRT).
- ``pin_sound_wave_decay``: Eqs. StressTensor and KinematicViscosity give a
  longitudinal viscosity 4 nu/3 + nu_B = nu + c_s^2 (tau_e - 1/2), so an
  isothermal sound wave of wave number k decays at
  k^2 (nu + c_s^2 (tau_e - 1/2)) / 2 per step.
"""
from __future__ import annotations

import numpy as np

import workloads as W
from tests.golden import mrt_matrix

C2 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
W2 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CS2 = 1.0 / 3.0


def _d3_velocities(orc):
    """The oracle's D3Q19 population order; the weights follow from |c|^2
    (1/3 at rest, 1/18 on the axes, 1/36 on the edges)."""
    c, _ = orc.d3q19_velocities()
    c2 = (c * c).sum(1)
    w = np.where(c2 == 0, 1 / 3, np.where(c2 == 1, 1 / 18, 1 / 36))
    return c, w


def _feq(c, w, rho, u):
    """Second-order equilibrium (Eq. EquilibriumDistribution), c_s^2 = 1/3.
    rho: field of shape S; u: list of D component fields of shape S."""
    uu = sum(ui * ui for ui in u)
    out = []
    for ci, wi in zip(c, w):
        cu = sum(int(ci[a]) * u[a] for a in range(len(u)))
        out.append(wi * rho * (1 + cu / CS2 + (cu * cu) / (2 * CS2 * CS2) - uu / (2 * CS2)))
    return np.array(out)


def _d1_feq(rho, u):
    return _feq(np.array([[0], [1], [-1]]), np.array([2 / 3, 1 / 6, 1 / 6]), rho, [u])


# ---------------------------------------------------------------------------
# (a) advection and conduction: exact amplification of a temperature mode
# ---------------------------------------------------------------------------
def _symbols(kind, k):
    """Closed-form symbols of the isotropic first and second differences of
    Sec. III (d_a phi = 3 sum_i w_i c_ia phi(x + c_i),
    lap phi = 6 sum_i w_i (phi(x + c_i) - phi(x))) on exp(i k.x).
    Returns (s, l) with d_a -> i s_a and lap -> l.

    Along an axis, on D1Q3, D2Q9 and D3Q19 alike: the weights of the
    velocities with c_a = +1 sum to 1/6, so s = sin k and l = 2 (cos k - 1).
    Along the D2Q9 diagonal k (1, 1): the axis links carry w = 1/9 with
    k.c = +-k, the diagonal links w = 1/36 with k.c in {+-2k, 0}, so
    s_x = s_y = (2/3) sin k + (1/6) sin 2k and
    l = (8/3)(cos k - 1) + (1/3)(cos 2k - 1)."""
    if kind == "axis":
        return np.sin(k), 2.0 * (np.cos(k) - 1.0)
    if kind == "diagonal":
        return (2 / 3) * np.sin(k) + (1 / 6) * np.sin(2 * k), \
            (8 / 3) * (np.cos(k) - 1) + (1 / 3) * (np.cos(2 * k) - 1)
    raise ValueError(kind)


TRANSPORT_CASES = [
    # lattice, shape (wall-normal axis first), wave vector in lattice units per axis of
    # shape, symbol kind, velocity, taus
    ("D1Q3", (16,), (1,), "axis", (0.05,), (1.0,) * 6),
    ("D2Q9", (3, 16), (0, 2), "axis", (0.01, 0.05), (1.0,) * 6),
    ("D2Q9", (16, 16), (1, 1), "diagonal", (0.03, 0.05), (1.0, 1.3, 0.9, 1.0, 1.2, 0.8)),
    ("D3Q19", (3, 1, 16), (0, 0, 1), "axis", (0.05, 0.02, -0.01), (1.0,) * 6),
    ("D3Q19", (16, 1, 1), (1, 0, 0), "axis", (0.0, 0.01, -0.04), (1.0,) * 6),
]


def pin_transport(orc, case, steps=200):
    lat, shape, modes, kind, u0, taus = case
    rho0, T0, A = 0.2, 1.0, 0.1
    kappa, cv = 0.02, 5.0
    if lat == "D1Q3":
        P = orc.make_params("D1Q3", ny=shape[0], walls=False, eos="ideal", kappa=kappa, cv=cv)
    elif lat == "D2Q9":
        P = orc.make_params("D2Q9", nx=shape[1], ny=shape[0], walls=False, eos="ideal",
                            kappa=kappa, cv=cv, tau=taus)
    else:
        P = orc.make_params("D3Q19", nx=shape[2], ny=shape[1], nz=shape[0], walls=False,
                            eos="ideal", kappa=kappa, cv=cv)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    kvec = [2 * np.pi * m / n for m, n in zip(modes, shape)]
    phase = sum(kk * g for kk, g in zip(kvec, grids))
    rho = np.full(shape, rho0)
    # velocity components in (x, y, z) order; the fields are indexed wall-normal first
    if lat == "D1Q3":
        f = _d1_feq(rho, np.full(shape, u0[0]))
        u_along = [u0[0]]
    elif lat == "D2Q9":
        f = _feq(C2, W2, rho, [np.full(shape, u0[0]), np.full(shape, u0[1])])
        u_along = [u0[1], u0[0]]  # (y, x) to match the shape order
    else:
        c, w = _d3_velocities(orc)
        f = _feq(c, w, rho, [np.full(shape, u) for u in u0])
        u_along = [u0[2], u0[1], u0[0]]
    f = np.ascontiguousarray(f).ravel()
    T = (T0 + A * np.cos(phase)).ravel().copy()
    orc.step(P, f, T, steps)
    # complex amplitude of exp(i k.x) in T - T0: (2/N) sum (T - T0) exp(-i k.x)
    amp = 2.0 * np.mean((T.reshape(shape) - T0) * np.exp(-1j * phase))
    k_along = max(kvec)
    s, l = _symbols(kind, k_along)
    udots = sum(u * s for u, kk in zip(u_along, kvec) if kk != 0)
    lam = -1j * udots + kappa * l / (rho0 * cv)
    G = 1 + lam + lam * lam / 2
    want = A * G ** steps
    assert abs(want) > 0.05 * A, "mode decayed too far to be a useful pin"
    err = abs(amp - want) / A
    assert err < 1e-12, (case, amp, want, err)
    # density and velocity stay uniform
    m = orc.macro(P, f, T)
    assert np.abs(m["rho"] - rho0).max() < 1e-15


# ---------------------------------------------------------------------------
# (b) pressure work: T follows rho adiabatically in a small density wave
# ---------------------------------------------------------------------------
WORK_CASES = [
    # lattice, shape (wall-normal axis first), axis of the wave in shape
    ("D1Q3", (64,), 0),
    ("D2Q9", (3, 64), 1),
    ("D3Q19", (3, 64, 1), 1),
]


def pin_adiabatic_work(orc, crit, case, steps=300):
    lat, shape, axis = case
    _, T_c, _ = crit
    T0, rho0, eps = 0.8 * T_c, 0.32, 1e-4
    kw = dict(walls=False, g=0.0, kappa=0.0)
    if lat == "D1Q3":
        P = orc.make_params("D1Q3", ny=shape[0], **kw)
    elif lat == "D2Q9":
        P = orc.make_params("D2Q9", nx=shape[1], ny=shape[0], **kw)
    else:
        P = orc.make_params("D3Q19", nx=shape[2], ny=shape[1], nz=shape[0], **kw)
    n = shape[axis]
    k = 2 * np.pi / n
    x = np.arange(n).reshape([-1 if a == axis else 1 for a in range(len(shape))])
    rho_init = np.broadcast_to(rho0 * (1 + eps * np.cos(k * x)), shape).copy()
    f = orc.init_rest(P, rho_init.ravel())
    T = np.full(rho_init.size, T0)
    basis = np.broadcast_to(np.exp(-1j * k * x), shape)

    def mode(a):
        return 2.0 * np.mean(a.reshape(shape) * basis)

    rho_start = orc.macro(P, f, T)["rho"].copy()
    eta0 = P.b * rho0 / 4
    Z0 = (1 + eta0 + eta0 ** 2 - eta0 ** 3) / (1 - eta0) ** 3
    coef = T0 * P.R * Z0 / (rho0 * P.cv)
    worst, scale = 0.0, 0.0
    prev = rho_start
    for _ in range(steps):
        orc.step(P, f, T, 1)
        rho = orc.macro(P, f, T)["rho"].copy()
        drho = mode(0.5 * (rho + prev) - rho_start)
        prev = rho
        dT = mode(T - T0)
        worst = max(worst, abs(dT - coef * drho))
        scale = max(scale, abs(coef * drho))
    # the wave must have moved the density for the pin to mean anything
    assert scale > 0.5 * coef * rho0 * eps, (case, scale)
    # left: the divergence symbol's k^2/6 (measured 1.5 k^2/6) and O(eps) nonlinear terms
    assert worst < 0.5 * k * k * scale, (case, worst / scale, k * k / 6)


# ---------------------------------------------------------------------------
# (c) D3Q19 on a slab equals D2Q9
# ---------------------------------------------------------------------------
def pin_d3q19_slab_equals_d2q9(orc, crit, form, orientation, steps=300, n_in=5, nz=14):
    _, T_c, _ = crit
    kw = dict(walls=True, g=2e-4, gravity_form=form, sigma=0.0, rho_v=0.05)
    P2 = orc.make_params("D2Q9", nx=n_in, ny=nz, **kw)
    # sigma = 0 drops Li's coexistence correction: 0.9 T_c keeps the interface stable
    rv, rl, _ = orc.coexistence(P2, 0.9 * T_c)
    rho0 = W.layered_density((nz, n_in), nz // 2, rl, rv, 0.0, seed=0)
    # vary the state along the in-plane axis too: a tilted, noisy interface
    tilt = 0.02 * np.cos(2 * np.pi * np.arange(n_in) / n_in)[None, :]
    rho0 = rho0 * (1 + tilt) * (1 + 1e-2 * W.uniform_pm1(61, rho0.size).reshape(rho0.shape))
    T0 = W.wall_temperature_field((nz, n_in), 0.9 * T_c, 0.93 * T_c, 0.88 * T_c)
    T0 = T0 * (1 + 1e-3 * np.sin(2 * np.pi * np.arange(n_in) / n_in)[None, :])
    f2 = orc.init_rest(P2, rho0.ravel())
    T2 = T0.ravel().copy()
    orc.step(P2, f2, T2, steps)
    m2 = orc.macro(P2, f2, T2)
    if orientation == "xz":
        P3 = orc.make_params("D3Q19", nx=n_in, ny=1, nz=nz, **kw)
        shape3 = (nz, 1, n_in)
    else:
        P3 = orc.make_params("D3Q19", nx=1, ny=n_in, nz=nz, **kw)
        shape3 = (nz, n_in, 1)
    f3 = orc.init_rest(P3, rho0.reshape(shape3).ravel())
    T3 = T0.reshape(shape3).ravel().copy()
    orc.step(P3, f3, T3, steps)
    m3 = orc.macro(P3, f3, T3)
    u_in = m3["ux"] if orientation == "xz" else m3["uy"]
    u_off = m3["uy"] if orientation == "xz" else m3["ux"]
    assert np.abs(m3["rho"] - m2["rho"]).max() < 1e-13 * rl, (form, orientation)
    assert np.abs(u_in - m2["ux"]).max() < 1e-14, (form, orientation)
    assert np.abs(m3["uz"] - m2["uy"]).max() < 1e-14, (form, orientation)
    assert np.abs(u_off).max() < 1e-16, (form, orientation)
    assert np.abs(T3 - T2).max() < 1e-13 * T_c, (form, orientation)


# ---------------------------------------------------------------------------
# (d) which moments each relaxation time acts on
# ---------------------------------------------------------------------------
RATE_OWNERS = {0: [], 1: [1], 2: [2], 3: [], 4: [4, 6], 5: [7, 8]}
TAU_NAMES = ("tau_rho", "tau_e", "tau_varsigma", "tau_j", "tau_q", "tau_nu")


def pin_relaxation_rate_mapping(orc, crit):
    _, T_c, _ = crit
    nx, ny = 4, 6
    base = (1.1, 0.9, 1.2, 0.8, 1.3, 0.7)
    rho0 = W.layered_density((ny, nx), 3, 0.28, 0.05, 0.05, seed=17)
    T = (0.8 * T_c * (1 + 0.01 * W.uniform_pm1(18, nx * ny)))
    M = mrt_matrix()
    P0 = orc.make_params("D2Q9", nx=nx, ny=ny, walls=False, g=3e-4, tau=base)
    f = orc.init_rest(P0, rho0.ravel()) * (1 + 0.03 * W.uniform_pm1(19, 9 * nx * ny))
    m_base = M @ orc.collide(P0, f, T).reshape(9, -1)
    for k, owners in RATE_OWNERS.items():
        taus = list(base)
        taus[k] = base[k] + 0.4
        P = orc.make_params("D2Q9", nx=nx, ny=ny, walls=False, g=3e-4, tau=taus)
        dm = np.abs(M @ orc.collide(P, f, T).reshape(9, -1) - m_base).max(axis=1)
        for j in range(9):
            if j in owners:
                assert dm[j] > 1e-6, (TAU_NAMES[k], j, dm[j])
            else:
                assert dm[j] < 1e-15, (TAU_NAMES[k], j, dm[j])


# ---------------------------------------------------------------------------
# (e) sound attenuation at the longitudinal viscosity
# ---------------------------------------------------------------------------
def pin_sound_wave_decay(orc, tau_e=1.3, tau_vs=0.7, tau_nu=0.8, L=64, skip=40, steps=400):
    taus = (1.0, tau_e, tau_vs, 1.0, 1.1, tau_nu)
    P = orc.make_params("D2Q9", nx=L, ny=3, walls=False, eos="ideal", g=0.0, tau=taus)
    k = 2 * np.pi / L
    x = np.arange(L)[None, :] * np.ones((3, 1))
    eps, rho0 = 1e-4, 1.0
    rho = rho0 * (1 + eps * np.cos(k * x))
    ux = np.sqrt(CS2) * eps * np.cos(k * x)  # a wave running towards +x
    f = np.ascontiguousarray(_feq(C2, W2, rho, [ux, np.zeros_like(ux)])).ravel()
    T = np.ones(rho.size)
    basis = np.exp(-1j * k * x)

    def amp():
        return abs(2.0 * np.mean(orc.macro(P, f, T)["rho"].reshape(3, L) * basis))

    orc.step(P, f, T, skip)
    t, a = [], []
    for s in range(0, steps + 1, 20):
        if s:
            orc.step(P, f, T, 20)
        t.append(s)
        a.append(np.log(amp()))
    rate = -np.polyfit(t, a, 1)[0]
    nu = CS2 * (tau_nu - 0.5)
    want = k * k * (nu + CS2 * (tau_e - 0.5)) / 2
    assert abs(rate / want - 1) < 2e-2, (rate, want)
