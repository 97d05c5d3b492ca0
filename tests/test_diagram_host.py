"""Host logic of the configuration-diagram sweep: morphology classification,
the lever-rule starts and their softening (no GPU needed)."""
import numpy as np
import pytest

from paper_2301_12869_amd import diagram as D

RV, RL = 0.0145, 0.333


@pytest.mark.parametrize("config", D.CONFIGS)
def test_sharp_starts_have_their_morphology_and_the_lever_rule_mass(config):
    mean = RV + 0.4 * (RL - RV)
    rho, faces = D.sharp_start(config, 101, mean, RV, RL)
    assert D.morphology(rho) == config
    assert len(faces) == (2 if config == "V-L-V" else 1)
    # liquid length as the lever rule puts it, to within one node
    n_liquid = np.count_nonzero(rho == RL)
    assert abs(n_liquid - 101 * 0.4) <= 1
    soft = D.soften(rho, faces, 2.0)
    assert D.morphology(soft) == config
    assert np.all(np.diff(soft[: int(faces[0]) - 8]) == 0)  # untouched away from the interfaces
    assert np.array_equal(D.soften(rho, faces, 0.0), rho)


def test_morphology_reads_phases_from_the_bottom():
    y = np.arange(60)
    assert D.morphology(np.where((y > 10) & (y < 30), RL, RV)) == "V-L-V"
    assert D.morphology(np.where((y < 10) | (y > 50), RL, RV)) == "L-V-L"
    assert D.morphology(np.full(60, 0.2) + 1e-3 * np.sin(y)) == "single"
    assert D.morphology(np.where(y < 59, RL, RV)) == "L-V"


def test_soften_is_monotone_across_an_interface():
    rho, faces = D.sharp_start("L-V", 81, RV + 0.5 * (RL - RV), RV, RL)
    soft = D.soften(rho, faces, 2.5)
    assert np.all(np.diff(soft) <= 0)
    assert soft[0] == RL and soft[-1] == RV
