"""The seeded input generators (shared by tests, benchmark and smoke check)."""
import numpy as np

import workloads as W


def test_splitmix64_reference_vector():
    # first outputs of the reference splitmix64.c generator seeded with 1234567
    assert list(map(int, W.splitmix64(1234567, 5))) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_counter_based_streams_are_position_independent():
    a = W.splitmix64(99, 20)
    b = W.splitmix64(99, 10, start=10)
    assert np.array_equal(a[10:], b)
    u = W.uniform_pm1(5, 100000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01


def test_layered_density_and_columns():
    r = W.layered_density((10, 4), 3, 0.3, 0.02, 0.0, seed=1)
    assert r.shape == (10, 4) and (r[:3] == 0.3).all() and (r[3:] == 0.02).all()
    r = W.layered_density((10, 4), 3, 0.3, 0.02, 1e-3, seed=1)
    assert np.abs(r[:3] / 0.3 - 1).max() <= 1e-3
    d = W.column_draws(4096, seed=3)
    assert d["height"].min() >= 128 and d["height"].max() <= 2048
    assert 1e-6 <= d["g"].min() and d["g"].max() <= 1e-4
    assert set(np.unique(d["form"])) == {1, 2}
    assert abs((d["form"] == 1).mean() - 0.5) < 0.05
    col = W.column_initial_density(200, 0.1, 0.3, 0.02, 0.0, 1)
    assert abs(col.mean() - 0.1) < 0.003
