"""The oracle's threaded node loops give bit for bit the serial results:
every node's arithmetic is unchanged, each output has one writer, and the
sums stay serial (D2Q9 with walls at general tau, both gravity forms;
D3Q19 with walls)."""
import numpy as np
import pytest

import workloads as W


def _run(orc, crit, lattice, form, threads):
    _, T_c, _ = crit
    prev = orc.set_threads(threads)
    try:
        if lattice == "D2Q9":
            shape = (40, 23)
            P = orc.make_params("D2Q9", nx=23, ny=40, g=1e-4, gravity_form=form,
                                tau=(1.0, 1.2, 0.9, 1.0, 1.1, 0.8))
        else:
            shape = (20, 6, 7)
            P = orc.make_params("D3Q19", nx=7, ny=6, nz=20, g=1e-4, gravity_form=form)
        rv, rl, _ = orc.coexistence(P, 0.8 * T_c)
        rho0 = W.layered_density(shape, shape[0] // 2, rl, rv, 1e-2, seed=71)
        T0 = W.wall_temperature_field(shape, 0.8 * T_c, 0.86 * T_c, 0.78 * T_c)
        f = orc.init_rest(P, rho0.ravel())
        T = T0.ravel().copy()
        d = orc.step(P, f, T, 60)
        return f, T, d
    finally:
        orc.set_threads(prev)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("form", [1, 2])
def test_threaded_oracle_is_bitwise_the_serial_oracle(orc, crit, lattice, form):
    f1, T1, d1 = _run(orc, crit, lattice, form, 1)
    f4, T4, d4 = _run(orc, crit, lattice, form, 4)
    assert np.array_equal(f1, f4)
    assert np.array_equal(T1, T4)
    assert d1 == d4
