"""Seeded synthetic workloads for the thermal pseudopotential LBM.

This module is shared by the tests, the benchmark and the smoke check, and it
holds none of the method's arithmetic: it only draws seeded random numbers and
lays out initial fields from numbers the caller supplies (coexistence
densities, temperatures, heights).  Whoever calls it computes those numbers
with its own equation-of-state code.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw ``i`` of stream ``seed`` is the SplitMix64 finaliser applied to
``seed + (i + 1) * 0x9E3779B97F4A7C15`` (mod 2^64).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+count-1 of the SplitMix64 stream of ``seed``."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed % (1 << 64)) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each draw."""
    return (splitmix64(seed, count, start) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform_pm1(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, count, start) - 1.0


# ---------------------------------------------------------------------------
# layered liquid / vapour states
# ---------------------------------------------------------------------------
def layered_density(shape, n_liquid: int, rho_l: float, rho_v: float, noise: float,
                    seed: int) -> np.ndarray:
    """Density field with liquid in the first ``n_liquid`` layers along the
    wall-normal axis (axis 0 of ``shape``, the slowest index) and vapour above,
    times (1 + noise * xi), xi uniform in [-1, 1) per node in linear index
    order.  ``shape`` is (ny,), (ny, nx) or (nz, ny, nx)."""
    shape = tuple(int(s) for s in shape)
    rho = np.full(shape, float(rho_v))
    rho[:n_liquid, ...] = float(rho_l)
    if noise:
        xi = uniform_pm1(seed, rho.size).reshape(shape)
        rho = rho * (1.0 + noise * xi)
    return np.ascontiguousarray(rho)


def wall_temperature_field(shape, T_bulk: float, T_bottom: float, T_top: float) -> np.ndarray:
    """Temperature field: bulk value everywhere, the first layer along the
    wall-normal axis at T_bottom and the last at T_top (the wall nodes keep
    these values as Dirichlet data)."""
    T = np.full(tuple(int(s) for s in shape), float(T_bulk))
    T[0, ...] = float(T_bottom)
    T[-1, ...] = float(T_top)
    return T


def linear_temperature_profile(n: int, T_bottom: float, T_top: float) -> np.ndarray:
    return np.linspace(float(T_bottom), float(T_top), int(n))


# ---------------------------------------------------------------------------
# the batched column sweep: raw seeded draws per column
# ---------------------------------------------------------------------------
def column_draws(n_cols: int, seed: int, h_min: int = 128, h_max: int = 2048,
                 log10_g=(-6.0, -4.0), t_reduced=(0.6, 0.95)) -> dict:
    """Raw per-column draws for a sweep of independent columns.

    Returns arrays of length n_cols:
      height     integer in [h_min, h_max] (nodes, both wall nodes included)
      g          10**U[log10_g]
      t_reduced  U[t_reduced]      (T / T_c; the caller multiplies by its T_c)
      form       1 or 2 with probability 1/2 each
      fill       U[0, 1)           (the caller maps it to a mean density
                                    between its vapour and liquid densities)
      seed       per-column noise seed
    """
    u = uniform01(seed, 6 * n_cols).reshape(n_cols, 6)
    height = h_min + np.minimum((u[:, 0] * (h_max - h_min + 1)).astype(np.int64),
                                h_max - h_min)
    g = 10.0 ** (log10_g[0] + (log10_g[1] - log10_g[0]) * u[:, 1])
    tr = t_reduced[0] + (t_reduced[1] - t_reduced[0]) * u[:, 2]
    form = np.where(u[:, 3] < 0.5, 1, 2).astype(np.int32)
    fill = u[:, 4]
    col_seed = (splitmix64(seed ^ 0x5DEECE66D, n_cols) >> np.uint64(1)).astype(np.int64)
    return dict(height=height.astype(np.int32), g=g, t_reduced=tr, form=form, fill=fill,
                seed=col_seed)


def column_initial_density(height: int, mean_rho: float, rho_l: float, rho_v: float,
                           noise: float, seed: int) -> np.ndarray:
    """Liquid below / vapour above a flat interface placed so that the
    layered profile has the requested mean (lever rule on node counts),
    times seeded noise.  The caller supplies rho_l, rho_v for its temperature."""
    frac = (mean_rho - rho_v) / (rho_l - rho_v)
    n_liq = int(round(frac * height))
    n_liq = max(0, min(height, n_liq))
    return layered_density((height,), n_liq, rho_l, rho_v, noise, seed)
