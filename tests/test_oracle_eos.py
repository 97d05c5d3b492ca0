"""Pins of the oracle's equation-of-state utilities (Sec. IV.B Eq. EOS,
Eq. MaxwellRule, spinodals of Sec. V) against things other than themselves:
finite differences of the raw pressure, numerical quadrature of the equal-area
integral, and the critical-constant relations the paper prints."""
import numpy as np
import pytest
from scipy import integrate

from tests.golden import paper_values

pytestmark = pytest.mark.filterwarnings("ignore")


def test_critical_point_is_an_inflection_with_zero_slope(orc, crit):
    rho_c, T_c, p_c = crit
    P = orc.make_params()
    h = 1e-5 * rho_c
    p = lambda r: orc.eos_p(P, r, T_c)  # noqa: E731
    d1 = (p(rho_c + h) - p(rho_c - h)) / (2 * h)
    d2 = (p(rho_c + h) - 2 * p(rho_c) + p(rho_c - h)) / h ** 2
    # scale: p_c / rho_c and p_c / rho_c^2
    assert abs(d1) < 1e-8 * p_c / rho_c
    assert abs(d2) < 1e-4 * p_c / rho_c ** 2
    # just below T_c there is a loop (negative slope at rho_c), just above none
    assert (orc.eos_p(P, rho_c + h, 0.999 * T_c) - orc.eos_p(P, rho_c - h, 0.999 * T_c)) < 0
    assert (orc.eos_p(P, rho_c + h, 1.001 * T_c) - orc.eos_p(P, rho_c - h, 1.001 * T_c)) > 0


def test_critical_constants_match_the_papers_approximations(crit):
    """Sec. IV.B prints a ~ 3.8533 p_c/rho_c^2, b ~ 0.5218/rho_c,
    R ~ 2.7864 p_c/(rho_c T_c) for the C-S EOS; with a=0.5, b=4, R=1 the
    oracle's exact critical point must reproduce them to the printed digits."""
    pv = paper_values()
    rho_c, T_c, p_c = crit
    assert pv["approx_a_coef"] * p_c / rho_c ** 2 == pytest.approx(pv["eos_a"], rel=3e-4)
    assert pv["approx_b_coef"] / rho_c == pytest.approx(pv["eos_b"], rel=3e-4)
    assert pv["approx_R_coef"] * p_c / (rho_c * T_c) == pytest.approx(pv["eos_R"], rel=3e-4)


def test_dpdT_and_dpdrho_against_finite_differences(orc, crit):
    rho_c, T_c, _ = crit
    P = orc.make_params()
    for rho in (0.01, 0.1, 0.3, 0.5):
        for tr in (0.6, 0.8, 1.1):
            T = tr * T_c
            hT = 1e-6 * T
            fd = (orc.eos_p(P, rho, T + hT) - orc.eos_p(P, rho, T - hT)) / (2 * hT)
            assert orc.eos_dpdT(P, rho, T) == pytest.approx(fd, rel=1e-8)
            hr = 1e-6 * rho
            fd = (orc.eos_p(P, rho + hr, T) - orc.eos_p(P, rho - hr, T)) / (2 * hr)
            assert orc.eos_dpdrho(P, rho, T) == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_low_density_limit_is_the_ideal_gas(orc):
    P = orc.make_params()
    rho, T = 1e-7, 0.04
    assert orc.eos_p(P, rho, T) == pytest.approx(rho * T, rel=1e-6)


@pytest.mark.parametrize("tr", [0.6, 0.7, 0.75, 0.8, 0.85, 0.9, 0.95])
def test_maxwell_equal_area_by_quadrature(orc, crit, tr):
    """Eq. MaxwellRule: equal pressures and zero area of (p_sat - p)/rho^2,
    the area evaluated by adaptive quadrature of the raw EOS."""
    _, T_c, p_c = crit
    P = orc.make_params()
    T = tr * T_c
    rv, rl, ps = orc.coexistence(P, T)
    sv, sl = orc.spinodal(P, T)
    assert 0 < rv < sv < sl < rl
    assert orc.eos_p(P, rv, T) == pytest.approx(ps, rel=1e-11)
    assert orc.eos_p(P, rl, T) == pytest.approx(ps, rel=1e-11, abs=1e-15)
    area, err = integrate.quad(lambda r: (ps - orc.eos_p(P, r, T)) / r ** 2, rv, rl,
                               points=[sv, sl], limit=400, epsabs=1e-14, epsrel=1e-13)
    scale = integrate.quad(lambda r: abs(ps - orc.eos_p(P, r, T)) / r ** 2, rv, rl,
                           points=[sv, sl], limit=400)[0]
    assert abs(area) < 1e-9 * scale


def test_spinodals_are_pressure_extrema(orc, crit):
    _, T_c, _ = crit
    P = orc.make_params()
    for tr in (0.6, 0.8, 0.95):
        T = tr * T_c
        for r in orc.spinodal(P, T):
            h = 1e-6 * r
            slope = (orc.eos_p(P, r + h, T) - orc.eos_p(P, r - h, T)) / (2 * h)
            assert abs(slope) < 1e-7
    with pytest.raises(RuntimeError):
        orc.spinodal(P, 1.01 * T_c)


def test_mean_density_reading_is_half_filled(orc, crit):
    """The paper's <rho> = 1.3344 (Sec. IV.B) read in units of rho_c lies
    within 0.2% of the Maxwell midpoint at T_med = 0.75 T_c: the reading gives
    a half-filled column, while 1.3344 in lattice units exceeds every liquid
    density of the model."""
    pv = paper_values()
    rho_c, T_c, _ = crit
    P = orc.make_params()
    rv, rl, _ = orc.coexistence(P, pv["T_med_reduced"] * T_c)
    assert pv["mean_rho_reduced"] * rho_c == pytest.approx(0.5 * (rv + rl), rel=2e-3)
    assert pv["mean_rho_reduced"] > rl


def test_pseudopotential_sign_reading(orc, crit):
    """With G = -1 the radicand 2(p - rho/3)/G of Eq. InteractionPotential is
    non-negative over the whole liquid-vapour range at lattice parameters."""
    _, T_c, _ = crit
    P = orc.make_params()
    for tr in (0.6, 0.8, 0.95):
        T = tr * T_c
        for rho in np.linspace(1e-4, 0.45, 50):
            assert 2 * (orc.eos_p(P, rho, T) - rho / 3) / -1.0 >= 0
