"""GPU parity of the warm-start network against its CPU reference.

The reference runs in FP64 with every product input rounded to bfloat16
(what a BF16 matrix core with FP32 accumulation computes, up to the order of
the FP32 sums).  The kernels differ from it only by FP32 rounding inside the
sums (relative ~1e-7 per sum of up to 320 terms) and by the rare BF16 rounding
of an intermediate that lands on the other side of a rounding boundary
because of it (one BF16 ulp, 2^-8 relative, of single elements).  Hence the
bounds: relative L2 error of outputs and of each layer's gradient below 2e-3,
and the kernels at least 10x closer to the BF16 reference than to the plain
FP64 network (so the test sees the BF16 arithmetic, not just a loose match).
"""
import numpy as np
import pytest

import workloads as W
from oracle import net_ref as N

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


@pytest.fixture(scope="module")
def consts(T):
    rho_c, T_c, _ = T.eos_critical(0.5, 4.0, 1.0)
    return rho_c, T_c


def _theta(seed):
    th = N.init_params(seed)
    th = th + 0.02 * W.uniform_pm1(seed + 1000, th.size)  # nonzero biases
    return th.astype(np.float32)


# (height, form, t_reduced, g, mean_reduced, lever_height): a 3-node column,
# ragged heights across the 32-position wave tiles and 128-position blocks,
# and the tallest column the sweep holds
COLS = [(37, 1, 0.8, 3e-5, 1.2, 15.3), (3, 2, 0.9, 1e-6, 0.7, 1.0), (130, 2, 0.72, 1e-4, 2.1, 77.7),
        (301, 1, 0.65, 7e-6, 1.6, 120.25), (64, 2, 0.95, 2e-5, 1.0, 40.0), (2048, 1, 0.85, 4e-6, 1.33, 1003.6)]


def _features(c):
    h, form, t, g, m, hl = c
    return N.features(h, t, g, form, m, hl)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _net(T, consts, max_cols=16, max_nodes=8192, dataset_cols=0, dataset_nodes=0):
    return T.Net(consts[0], consts[1], max_cols=max_cols, max_nodes=max_nodes,
                 dataset_cols=dataset_cols, dataset_nodes=dataset_nodes)


def test_mfma_lane_layout(T, consts):
    """One 32x32x16 BF16 product on small integers (exact in FP32) against
    the lane layout the kernels assume: A[i][k] in lane i + 32 (k / 8),
    element k % 8; B[k][j] likewise with j; D[row][col] in lane col + 32 q,
    element r with row = 8 (r / 4) + 4 q + r % 4."""
    net = _net(T, consts)
    ra = np.round(4 * W.uniform_pm1(1, 512)).astype(np.float32)
    rb = np.round(4 * W.uniform_pm1(2, 512)).astype(np.float32)
    a16 = (ra.view(np.uint32) >> 16).astype(np.uint16)
    b16 = (rb.view(np.uint32) >> 16).astype(np.uint16)
    A = np.zeros((32, 16)); B = np.zeros((16, 32))
    for lane in range(64):
        for e in range(8):
            k = 8 * (lane // 32) + e
            A[lane % 32, k] = ra[8 * lane + e]
            B[k, lane % 32] = rb[8 * lane + e]
    D = A @ B
    d = net.mfma_check(a16, b16)
    for lane in range(64):
        for r in range(16):
            row = 8 * (r // 4) + 4 * (lane // 32) + r % 4
            assert d[lane, r] == D[row, lane % 32], (lane, r)
    net.close()


def test_forward_matches_the_bf16_reference(T, consts):
    theta = _theta(5)
    net = _net(T, consts)
    net.set_params(theta)
    got = net.forward(COLS)
    k = 0
    for c in COLS:
        h = c[0]
        x = _features(c)
        ref, _ = N.forward(theta.astype(np.float64), x, use_bf16=True)
        ref64, _ = N.forward(theta.astype(np.float64), x, use_bf16=False)
        g = got[k:k + h].T
        k += h
        e, e64 = _rel(g, ref), _rel(g, ref64)
        _log(f"column {c}: rel err vs bf16 ref {e:.2e}, vs fp64 ref {e64:.2e}")
        assert e < 2e-3
        assert e < 0.1 * e64 or e < 1e-5
    net.close()


def _dataset(consts, cols, seed):
    rho_c, T_c = consts
    tg, rho, TT = [], [], []
    k = 0
    rng = W.uniform_pm1(seed, sum(2 * c[0] for c in cols))
    for c in cols:
        h, form, t, g, m, hl = c
        tgt = 0.3 * rng[k:k + 2 * h].reshape(2, h)
        k += 2 * h
        tg.append(tgt)
        rho.append(rho_c * (tgt[0] + m))
        TT.append(T_c * (tgt[1] + t))
    # the reference sees the targets the kernels form from the profiles
    tg = [np.vstack([r / rho_c - c[4], t / T_c - c[2]]) for r, t, c in zip(rho, TT, cols)]
    return tg, np.concatenate(rho), np.concatenate(TT)


def test_gradient_matches_the_bf16_reference(T, consts):
    cols = COLS[:5]
    theta = _theta(7)
    tg, rho, TT = _dataset(consts, cols, 8)
    n = sum(c[0] for c in cols)
    net = _net(T, consts, dataset_cols=len(cols), dataset_nodes=n)
    net.set_params(theta)
    net.set_dataset(cols, rho, TT)
    idx = np.arange(len(cols))
    L, g = net.loss_grad(idx)
    xs = [_features(c) for c in cols]
    Lr, gr = N.loss_and_grad(theta.astype(np.float64), xs, tg, use_bf16=True)
    L64, g64 = N.loss_and_grad(theta.astype(np.float64), xs, tg, use_bf16=False)
    _log(f"loss gpu {L:.8e} ref {Lr:.8e}")
    assert L == pytest.approx(Lr, rel=1e-4)
    Ws, bs = N.unflatten(np.arange(theta.size))
    for l in range(N.N_LAYERS):
        for name, sel in (("W", Ws[l].ravel()), ("b", bs[l].ravel())):
            e, e64 = _rel(g[sel], gr[sel]), _rel(g[sel], g64[sel])
            _log(f"layer {l} d{name}: rel err vs bf16 ref {e:.2e}, vs fp64 ref {e64:.2e}")
            assert e < 2e-3, (l, name)
    assert _rel(g, gr) < 0.1 * _rel(g, g64)
    # a second call is bitwise identical (fixed-order reductions)
    L2, g2 = net.loss_grad(idx)
    assert L2 == L and np.array_equal(g2, g)
    net.close()


def test_large_batch_gradient_equals_the_mean_of_its_columns(T, consts):
    """A 64 x 2048-position batch gives the weight-gradient kernel slices of
    at least 512 positions, which it stages in 128-position chunks; its
    gradient must equal the mean of its columns' gradients taken one column
    at a time (64-position chunks, the path the reference test pins), up to
    the order of the FP32 sums.  Equal heights put the per-column loss scale
    a power of two (64) from the batch's, so dZ rounds to BF16 alike."""
    nc, h = 64, 2048
    cols = [(h, 1 + k % 2, 0.7 + 0.2 * k / nc, 10 ** (-6 + 2 * k / nc), 0.8 + k / nc, h / 2) for k in range(nc)]
    theta = _theta(11)
    tg, rho, TT = _dataset(consts, cols, 12)
    net = _net(T, consts, max_cols=nc, max_nodes=nc * h, dataset_cols=nc, dataset_nodes=nc * h)
    net.set_params(theta)
    net.set_dataset(cols, rho, TT)
    L, g = net.loss_grad(np.arange(nc))
    acc, Ls = np.zeros(g.size), 0.0
    for k in range(nc):
        Lk, gk = net.loss_grad([k])
        acc += gk.astype(np.float64)
        Ls += Lk
    acc /= nc
    Ls /= nc
    _log(f"batch loss {L:.10e}, mean of columns {Ls:.10e}")
    assert L == pytest.approx(Ls, rel=1e-6)
    Ws, bs = N.unflatten(np.arange(theta.size))
    for l in range(N.N_LAYERS):
        for name, sel in (("W", Ws[l].ravel()), ("b", bs[l].ravel())):
            e = _rel(g[sel].astype(np.float64), acc[sel])
            _log(f"layer {l} d{name}: batch vs mean of columns {e:.2e}")
            assert e < 1e-4, (l, name)
    net.close()


def test_adam_step_matches_the_reference_and_training_lowers_the_loss(T, consts):
    cols = [(96, 1, 0.8, 1e-5, 1.3, 40.0), (200, 2, 0.7, 5e-5, 1.1, 60.5), (57, 1, 0.9, 2e-6, 1.5, 30.0)]
    theta = _theta(9)
    tg, rho, TT = _dataset(consts, cols, 10)
    n = sum(c[0] for c in cols)
    net = _net(T, consts, dataset_cols=len(cols), dataset_nodes=n)
    net.set_params(theta)
    net.set_dataset(cols, rho, TT)
    idx = np.arange(len(cols))
    _, g = net.loss_grad(idx)
    lr = 1e-3
    net.train_step(idx, lr)
    got = net.get_params()
    want, _, _ = N.adam_step(theta.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr)
    assert np.abs(got - want).max() < 1e-6
    # a smooth target the network can fit: loss falls by 10x within 300 steps
    rho_c, T_c = consts
    rho_s, T_s = [], []
    for (h, form, t, gg, m, hl) in cols:
        s = (np.arange(h) + 0.5) / h
        rho_s.append(rho_c * (m + 0.5 * np.tanh((0.4 - s) * 20)))
        T_s.append(np.full(h, T_c * t))
    net.set_params(theta)
    net.set_dataset(cols, np.concatenate(rho_s), np.concatenate(T_s))
    first = net.train_step(idx, 2e-3)
    for _ in range(300):
        last = net.train_step(idx, 2e-3)
    _log(f"training loss {first:.3e} -> {last:.3e}")
    assert last < 0.1 * first
    net.close()


def test_predict_keeps_the_mean_density_and_the_wall_temperatures(T, consts):
    rho_c, T_c = consts
    theta = _theta(11)
    net = _net(T, consts)
    net.set_params(theta)
    raw = net.forward(COLS)
    rho, TT = net.predict(COLS)
    k = 0
    for (h, form, t, g, m, hl) in COLS:
        r, tt, o = rho[k:k + h], TT[k:k + h], raw[k:k + h].astype(np.float64)
        k += h
        assert r.mean() == pytest.approx(m * rho_c, rel=1e-13)
        assert tt[0] == T_c * t and tt[-1] == T_c * t
        base = rho_c * (o[:, 0] + m)
        shift = m * rho_c - base.mean()
        np.testing.assert_allclose(r, base + shift, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(tt[1:-1], T_c * (t + o[1:-1, 1]), rtol=1e-13)
    net.close()


def test_bad_arguments_are_rejected(T, consts):
    net = _net(T, consts, max_cols=2, max_nodes=100)
    with pytest.raises(T.TplbmError):
        net.forward([(10, 1, 0.8, 1e-5, 1.3, 5.0)])  # parameters not set yet
    net.set_params(_theta(1))
    with pytest.raises(T.TplbmError):
        net.forward([(60, 1, 0.8, 1e-5, 1.3, 5.0), (60, 1, 0.8, 1e-5, 1.3, 5.0)])  # 120 nodes > 100
    with pytest.raises(T.TplbmError):
        net.forward([(10, 3, 0.8, 1e-5, 1.3, 5.0)])  # gravity form
    with pytest.raises(T.TplbmError):
        net.forward([(10, 1, 0.8, -1e-5, 1.3, 5.0)])  # g <= 0
    with pytest.raises(T.TplbmError):
        net.train_step([0], 1e-3)  # no dataset
    bad = _theta(1)
    bad[5] = np.nan
    with pytest.raises(T.TplbmError):
        net.set_params(bad)
    net.close()


def test_c_initialisation_equals_the_reference_draw(T, consts):
    """tplbm_net_init(seed) draws the He-uniform weights of the reference's
    init_params (same SplitMix64 stream, same order, rounded to FP32) and
    zero biases, bit for bit."""
    rho_c, T_c = consts
    net = T.Net(rho_c, T_c, max_cols=4, max_nodes=256)
    for seed in (0, 12345, 2 ** 63 + 7):
        net.init(seed)
        got = net.get_params()
        want = N.init_params(seed).astype(np.float32)
        assert np.array_equal(got, want), seed
    net.close()


def test_device_prediction_equals_the_host_prediction(T, consts):
    """tplbm_net_predict_device writes the same profiles into device arrays."""
    import torch

    rho_c, T_c = consts
    net = T.Net(rho_c, T_c, max_cols=len(COLS), max_nodes=sum(c[0] for c in COLS))
    net.set_params(_theta(11))
    rho, Tp = net.predict(COLS)
    n = rho.size
    dr = torch.empty(n, dtype=torch.float64, device=net.device)
    dT = torch.empty(n, dtype=torch.float64, device=net.device)
    net.predict_device(COLS, dr, dT)
    torch.cuda.synchronize()
    assert np.array_equal(dr.cpu().numpy(), rho)
    assert np.array_equal(dT.cpu().numpy(), Tp)
    with pytest.raises(ValueError):
        net.predict_device(COLS, dr[:-1], dT)
    net.close()
