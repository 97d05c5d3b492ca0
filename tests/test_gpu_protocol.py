"""Phase-change protocol (Sec. V A) on the batched sweep: equilibrate with
the top wall at 0.6213 T_c, then cool it to the target.  At the paper's first
case (T_bot = 0.9083 T_c, T_top = 0.5917 T_c, dT/T_c = 0.3166) the paper's
lattice keeps its liquid at the bottom, and so does this one.  At
dT/T_c = 0.35 with T_med = 0.75 T_c (past the paper's lattice limit of 0.3382;
T_bot = 0.925 T_c) the liquid at the bottom wall boils: in this lattice
already during the first stage, whose bottom wall is that hot too."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    from paper_2301_12869_amd import protocol as P

    return P


def test_the_papers_first_case_keeps_its_liquid(P):
    print("protocol: T_bot 0.9083, dT 0.3166, 5e5 steps after the change", flush=True)
    (r,) = P.boiling_scan([0.3166], second_steps=500_000, log=lambda m: print(m, flush=True))
    print(r, flush=True)
    assert r["first_stage"]["status"] == "converged"
    assert r["vapour_layer_at"] is None and r["diverged_at"] is None and r["final"] == "L-V"


def test_a_larger_difference_grows_vapour_at_the_bottom_wall(P):
    print("protocol: T_med 0.75, dT 0.35, 5e5 steps after the change", flush=True)
    (r,) = P.boiling_scan([0.35], t_bot=None, second_steps=500_000, log=lambda m: print(m, flush=True))
    print(r, flush=True)
    assert r["diverged_at"] is None
    assert r["first_stage"]["final"].startswith("V") or r["vapour_layer_at"] is not None
    assert r["final"].startswith("V")
