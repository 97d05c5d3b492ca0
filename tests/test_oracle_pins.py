"""The oracle against the pins of tests/oracle_pins.py (energy transport,
pressure work, D3Q19 isotropy and wall terms, relaxation-rate mapping,
longitudinal viscosity).  What each pin fixes is stated there."""
import pytest

from tests import oracle_pins as P


@pytest.mark.parametrize("case", P.TRANSPORT_CASES, ids=lambda c: f"{c[0]}-{c[3]}-{len(c[1])}d")
def test_temperature_mode_follows_the_heun_amplification(orc, case):
    P.pin_transport(orc, case)


@pytest.mark.parametrize("case", P.WORK_CASES, ids=lambda c: c[0])
def test_pressure_work_couples_temperature_to_density_adiabatically(orc, crit, case):
    P.pin_adiabatic_work(orc, crit, case)


@pytest.mark.parametrize("orientation", ["xz", "yz"])
@pytest.mark.parametrize("form", [1, 2, 3])
def test_d3q19_slab_equals_d2q9_at_sigma_zero(orc, crit, form, orientation):
    P.pin_d3q19_slab_equals_d2q9(orc, crit, form, orientation)


def test_each_relaxation_time_acts_on_its_own_moments(orc, crit):
    P.pin_relaxation_rate_mapping(orc, crit)


@pytest.mark.parametrize("tau_e,tau_vs", [(1.3, 0.7), (0.8, 1.4)])
def test_sound_wave_decays_at_the_longitudinal_viscosity(orc, tau_e, tau_vs):
    P.pin_sound_wave_decay(orc, tau_e=tau_e, tau_vs=tau_vs)
