"""Reference of the warm-start network (numpy, FP64).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU leg call it; the
product's HIP kernels never use it.

The network maps a column's parameters to its steady profiles.  Input at
position y of a column of height H (channels, in this order):
    s - 1/2 with s = (y + 1/2)/H,  T/T_c - 0.8,  log10(g) + 5,  form - 3/2,
    <rho>/rho_c - 1.3,  H/2048 - 1/2,  clip(d/32, -4, 4)/4,  clip(d/4, -4, 4)/4
with d = y + 1/2 - h the distance (in nodes) to the lever-rule interface
height h = H (<rho> - rho_v)/(rho_l - rho_v) of the column (rho_v, rho_l:
Maxwell coexistence densities at T; the caller computes h).  The last two
channels locate the interface to a fraction of a node even in BF16, which
the coarse position channel cannot do for tall columns (8-bit mantissa).
Six 1-D convolutions of width 5 with zero padding at both ends of the column
(the column never sees its neighbours in a batch), ReLU after the first five:
    8 -> 64 -> 64 -> 64 -> 64 -> 64 -> 2.
Output channels: rho/rho_c - <rho>/rho_c and T/T_c - T_wall/T_c.
Loss: mean over positions and both channels of the squared error.

Weights are W[l] with shape (C_out, 5, C_in) (tap-major in the middle, so tap
t reads the input at y + t - 2) and biases b[l] (C_out,).  With
bf16=True the inputs of every product (activations, weights, and the
back-propagated gradients entering a product) are rounded to bfloat16
(round to nearest even) first while sums stay exact, which is what a BF16
matrix core with FP32 accumulation computes up to the accumulation order.
"""
from __future__ import annotations

import numpy as np

CHANNELS = [8, 64, 64, 64, 64, 64, 2]
TAPS = 5
N_LAYERS = 6


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(height: int, t_reduced: float, g: float, form: int, mean_reduced: float,
             lever_height: float) -> np.ndarray:
    """Input channels (8, H) of one column."""
    H = int(height)
    y = np.arange(H) + 0.5
    s = y / H
    d = y - lever_height
    x = np.zeros((8, H))
    x[0] = s - 0.5
    x[1] = t_reduced - 0.8
    x[2] = np.log10(g) + 5.0
    x[3] = form - 1.5
    x[4] = mean_reduced - 1.3
    x[5] = H / 2048.0 - 0.5
    x[6] = np.clip(d / 32.0, -4.0, 4.0) / 4.0
    x[7] = np.clip(d / 4.0, -4.0, 4.0) / 4.0
    return x


def param_shapes():
    out = []
    for l in range(N_LAYERS):
        out.append(((CHANNELS[l + 1], TAPS, CHANNELS[l]), (CHANNELS[l + 1],)))
    return out


def n_params() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unflatten(theta: np.ndarray):
    Ws, bs, k = [], [], 0
    for ws, bsh in param_shapes():
        n = int(np.prod(ws))
        Ws.append(theta[k:k + n].reshape(ws))
        k += n
        n = int(np.prod(bsh))
        bs.append(theta[k:k + n].reshape(bsh))
        k += n
    return Ws, bs


def flatten(Ws, bs) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)])


def _conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[o, p] = b[o] + sum_{t, i} W[o, t, i] x[i, p + t - 2], zero outside."""
    C_in, H = x.shape
    xp = np.zeros((C_in, H + 4))
    xp[:, 2:2 + H] = x
    y = np.repeat(b[:, None], H, axis=1).astype(np.float64)
    for t in range(TAPS):
        y = y + W[:, t, :] @ xp[:, t:t + H]
    return y


def forward(theta: np.ndarray, x: np.ndarray, use_bf16: bool = False):
    """Returns the output (2, H) and the list of layer inputs (for backward)."""
    Ws, bs = unflatten(theta)
    acts = []
    a = x
    for l in range(N_LAYERS):
        ai = bf16(a) if use_bf16 else a
        Wl = bf16(Ws[l]) if use_bf16 else Ws[l]
        acts.append(ai)
        z = _conv(ai, Wl, bs[l])
        a = np.maximum(z, 0.0) if l < N_LAYERS - 1 else z
    return a, acts


def loss_and_grad(theta: np.ndarray, xs, targets, use_bf16: bool = False):
    """Mean squared error over all positions and both output channels of a
    batch of columns (lists of (8, H) inputs and (2, H) targets), and its
    gradient with respect to theta."""
    Ws, bs = unflatten(theta)
    total = sum(x.shape[1] for x in xs) * 2
    L = 0.0
    gW = [np.zeros_like(W) for W in Ws]
    gb = [np.zeros_like(b) for b in bs]
    for x, tgt in zip(xs, targets):
        out, acts = forward(theta, x, use_bf16)
        r = out - tgt
        L += float((r * r).sum())
        d = 2.0 * r / total  # dL/d(out)
        H = x.shape[1]
        for l in range(N_LAYERS - 1, -1, -1):
            # d: gradient w.r.t. the layer's pre-activation z
            dz = d
            db = dz.sum(axis=1)
            a = acts[l]
            ap = np.zeros((a.shape[0], H + 4))
            ap[:, 2:2 + H] = a
            dzq = bf16(dz) if use_bf16 else dz
            for t in range(TAPS):
                gW[l][:, t, :] += dzq @ ap[:, t:t + H].T
            gb[l] += db
            if l == 0:
                break
            # gradient w.r.t. the layer input a = relu(z_prev)
            Wl = bf16(Ws[l]) if use_bf16 else Ws[l]
            dp = np.zeros((dz.shape[0], H + 4))
            dp[:, 2:2 + H] = dzq
            da = np.zeros_like(a)
            for t in range(TAPS):
                # a[i, p] feeds z[o, p - t + 2]
                da += Wl[:, t, :].T @ dp[:, 4 - t:4 - t + H]
            d = da * (a > 0)
    return L / total, flatten(gW, gb)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights from the shared seeded generator, zero biases."""
    import workloads as W

    parts, k = [], 0
    for ws, bsh in param_shapes():
        fan_in = ws[1] * ws[2]
        lim = np.sqrt(6.0 / fan_in)
        n = int(np.prod(ws))
        parts.append(lim * W.uniform_pm1(seed, n, start=k))
        k += n
        parts.append(np.zeros(int(np.prod(bsh))))
    return np.concatenate(parts)


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) with bias-corrected moments; t is
    the 1-based step number.  Returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
