"""Host-side logic of the warm-start pipeline (no GPU): the column draw, the
parameter initialisation and the morphology count used to compare steady
states."""
import numpy as np

from paper_2301_12869_amd import warmstart as WS


def test_interface_count():
    s = np.linspace(0, 1, 200)
    lv = 0.3 - 0.28 * (np.tanh((s - 0.4) * 40) + 1) / 2          # liquid below vapour
    vlv = 0.02 + 0.28 * np.exp(-((s - 0.5) / 0.1) ** 8)            # vapour, liquid slab, vapour
    assert WS.interfaces(lv) == 1
    assert WS.interfaces(vlv) == 2
    assert WS.interfaces(lv[::-1]) == 1


def test_column_draw_and_parameters():
    c = WS.Columns(64, 5)
    assert c.rho0.size == c.height.sum() == c.offsets[-1]
    assert ((c.height >= 128) & (c.height <= 2048)).all()
    assert set(np.unique(c.form)) <= {1, 2}
    # the recorded mean is the exact mean of each plain start, in units of rho_c
    k = 7
    r = c.rho0[c.offsets[k]:c.offsets[k + 1]]
    assert abs(r.mean() / c.rho_c - c.mean_reduced[k]) < 1e-14
    # liquid below vapour
    assert r[: len(r) // 20].mean() > r[-len(r) // 20:].mean()
    nc = c.net_columns([k])[0]
    assert nc[0] == c.height[k] and nc[2] == c.t_reduced[k]
    th = WS.init_params(3)
    assert th.dtype == np.float32 and th.size == 85442
    # biases start at zero, weights inside the He-uniform bound of layer 0
    assert np.all(th[2560:2624] == 0) and np.abs(th[:2560]).max() <= np.sqrt(6 / 40)


def test_lever_rule_height():
    """The lever-rule height puts the mean density's mass into a flat
    liquid-below-vapour profile: H <rho> = h rho_l + (H - h) rho_v."""
    from paper_2301_12869_amd import eos_coexistence

    c = WS.Columns(16, 9)
    for k in range(16):
        H, h = c.height[k], c.lever_height[k]
        rv, rl, _ = eos_coexistence(c.t_reduced[k] * c.T_c)
        assert 0.0 <= h <= H
        assert abs(h * rl + (H - h) * rv - H * c.mean_reduced[k] * c.rho_c) < 1e-12 * H
