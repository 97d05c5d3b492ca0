"""Sharp-interface theoretical solution of a 1-D column (Sec. IV A and the
appendix on its numerical procedure) -- reference implementation.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark call it; the product's
code never does.

At rest (u = 0) the column obeys dp/dy = F_g,y(rho) (Eq. Momentum_Balance_TS)
and -kappa dT/dy = q' (Eq. Energy_TS); with constant kappa T is linear
between the wall temperatures (Eq. Temp_Profile).  Interfaces are sharp: at
an interface at height h_i the two phases have the Maxwell coexistence
densities and pressure of T(h_i) (Eqs. Integral_MaxwellRule and
Pressures_MaxwellRule).  Away from it the pressure is advanced with explicit
Euler steps, p(y + dy) = p(y) + F(rho(y)) dy, and the density follows from
the inverse EOS on the stable or metastable branch of the phase
(Eqs. Inverse_EOS, Numerical_Vapor_Region, Numerical_Liquid_Region).  A
branch pushed past its spinodal, or a vapour pushed to zero pressure, means
the configuration does not exist.  The interface height is varied until the
mean density equals the given <rho> (Sec. IV A, Sec. VI).

Configurations (Sec. VI): "L-V" liquid below vapour; "V-L" the same with the
phases swapped; "V-L-V" solved as V-L until the liquid pressure meets the
local saturation pressure, where a second interface starts a vapour phase.

Geometry (the lattice's): H nodes y = 0 .. H-1, the walls on nodes 0 and H-1,
T(y) = T_bot + (T_top - T_bot) y / (H - 1), y up, g > 0 pointing down,
F = -rho g (form 1), -(rho - <rho>) g (form 2) or -(rho - rho_v) g with a
given rho_v (form 3, Eq. Gravity_3).

Readings where the paper leaves the details open:
  * Euler steps: each node interval is split into `m` equal steps; the
    interval holding an interface is split at the interface, and each part
    into `m` steps.  A second interface (V-L-V) is placed inside the Euler
    step where p - p_sat changes sign, by linear interpolation of that
    difference; the vapour restarts there at the coexistence state.
  * Mass: the mean density is the integral of the sharp profile over the H
    node cells [-1/2, H - 1/2] divided by H -- the trapezoidal integral over
    the Euler steps between the walls plus half a cell at each wall holding
    the wall value.  For a smooth profile this is the node mean; across an
    interface it is continuous in h_i, so the search can bisect on it.
  * Search: the interface is placed on every node 0 .. H-1 in turn; the
    first pair of neighbouring placements that both exist and bracket
    <rho> is bisected to a width of 1e-12 (the lowest root, for the V-L-V
    case whose mean need not be monotone in h_i).
  * A node exactly on an interface takes the lower phase's value.
  * Above T_c the EOS has one branch; an interface cannot lie there.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O

CONFIGS = ("L-V", "V-L", "V-L-V")


class NoSolution(Exception):
    pass


def inverse_eos(P, p, T, branch, Tc, guess=None):
    """rho with p_EOS(rho, T) = p on branch 'v' (0 < rho <= vapour spinodal)
    or 'l' (liquid spinodal <= rho < 4/b); above T_c the one branch.
    Safeguarded Newton: Newton steps inside a bisection bracket on the
    monotone branch."""
    pole = 4.0 / P.b
    if T >= Tc:
        if p <= 0.0:
            raise NoSolution("zero pressure")
        lo, hi = 0.0, pole
    elif branch == "v":
        sv, _ = O.spinodal(P, T)
        if p <= 0.0:
            raise NoSolution("zero pressure")
        if p > O.eos_p(P, sv, T):
            raise NoSolution("vapour spinodal")
        lo, hi = 0.0, sv
    else:
        _, sl = O.spinodal(P, T)
        if p < O.eos_p(P, sl, T):
            raise NoSolution("liquid spinodal")
        lo, hi = sl, pole
    x = guess if guess is not None and lo < guess < hi else 0.5 * (lo + hi)
    for _ in range(200):
        f = O.eos_p(P, x, T) - p
        if f == 0.0:
            return x
        if f > 0.0:
            hi = x
        else:
            lo = x
        d = O.eos_dpdrho(P, x, T)
        xn = x - f / d if d > 0.0 else 0.5 * (lo + hi)
        if not (lo < xn < hi):
            xn = 0.5 * (lo + hi)
        if abs(xn - x) <= 1e-15 * x or hi - lo <= 1e-15 * hi:
            return xn
        x = xn
    return x


class Column:
    """One column's theoretical equilibrium (see the module docstring)."""

    def __init__(self, P, H, T_bot, T_top, g, form, mean, m=8, rho_v=0.0):
        if H < 3 or form not in (1, 2, 3) or m < 1:
            raise ValueError("bad column")
        self.P, self.H, self.T_bot, self.T_top = P, int(H), float(T_bot), float(T_top)
        self.g, self.form, self.mean, self.m = float(g), int(form), float(mean), int(m)
        self.rho_v = float(rho_v)
        self.Tc = O.critical(P.a, P.b, P.R)[1]

    def T(self, y):
        return self.T_bot + (self.T_top - self.T_bot) * y / (self.H - 1)

    def F(self, rho):
        """F_g,y of Eqs. Gravity_1 / Gravity_2 / Gravity_3 with y up."""
        if self.form == 2:
            return -(rho - self.mean) * self.g
        if self.form == 3:
            return -(rho - self.rho_v) * self.g
        return -rho * self.g

    def psat(self, y):
        return O.coexistence(self.P, self.T(y))[2]

    def _march(self, y0, p0, rho0, branch, up, watch_saturation=False):
        """Euler march from the state (y0, p0, rho0) towards the top (up) or
        bottom wall.  Returns (nodes, integral, switch): node -> (rho, p) for
        the nodes it passes (a node at y0 itself included), the trapezoidal
        integral of rho over the span it covered, and, if watch_saturation,
        the (y, p) where p - p_sat first changed sign (None if never)."""
        nodes, integral = {}, 0.0
        y, p, rho = y0, p0, rho0
        d_prev = 0.0
        if watch_saturation:
            d_prev = p - self.psat(y) if self.T(y) < self.Tc else 0.0
        node = math.ceil(y0) if up else math.floor(y0)
        end = self.H - 1 if up else 0
        while (node <= end) if up else (node >= end):
            step = (node - y) / self.m
            if step != 0.0:
                for _ in range(self.m):
                    p_new = p + self.F(rho) * step
                    y_new = y + step
                    if watch_saturation and self.T(y_new) < self.Tc:
                        d_new = p_new - self.psat(y_new)
                        if d_prev != 0.0 and (d_new == 0.0 or (d_new > 0.0) != (d_prev > 0.0)):
                            s = d_prev / (d_prev - d_new)
                            ys = y + s * step
                            ps = p + s * (p_new - p)
                            rs = inverse_eos(self.P, ps, self.T(ys), branch, self.Tc, rho)
                            integral += 0.5 * (rho + rs) * abs(ys - y)
                            return nodes, integral, (ys, ps)
                        d_prev = d_new
                    rho_new = inverse_eos(self.P, p_new, self.T(y_new), branch, self.Tc, rho)
                    integral += 0.5 * (rho + rho_new) * abs(step)
                    y, p, rho = y_new, p_new, rho_new
            y = float(node)
            nodes[node] = (rho, p)
            node += 1 if up else -1
        return nodes, integral, None

    def profile(self, config, h):
        """(rho, p, mean, interfaces) for configuration `config` with its
        (lower) interface at height h; raises NoSolution if it cannot exist."""
        if config not in CONFIGS:
            raise ValueError(config)
        if not 0.0 <= h <= self.H - 1:
            raise ValueError("interface outside the column")
        Ti = self.T(h)
        if Ti >= self.Tc:
            raise NoSolution("interface above T_c")
        rv, rl, ps = O.coexistence(self.P, Ti)
        if config == "L-V":
            lower, upper = ("l", rl), ("v", rv)
        else:
            lower, upper = ("v", rv), ("l", rl)
        down, i_down, _ = self._march(h, ps, lower[1], lower[0], up=False)
        up, i_up, switch = self._march(h, ps, upper[1], upper[0], up=True,
                                       watch_saturation=(config == "V-L-V"))
        interfaces = [h]
        pieces = [(lambda k: k <= h, down), (lambda k: k > h, up)]
        integral = i_down + i_up
        if config == "V-L-V":
            if switch is None:
                raise NoSolution("the liquid never meets the saturation pressure")
            y2 = switch[0]
            rv2, _, ps2 = O.coexistence(self.P, self.T(y2))
            top, i_top, _ = self._march(y2, ps2, rv2, "v", up=True)
            integral += i_top
            interfaces.append(y2)
            pieces = [(lambda k: k <= h, down), (lambda k: h < k < y2, up), (lambda k: k >= y2, top)]
        last = top if config == "V-L-V" else up
        rho, p = np.empty(self.H), np.empty(self.H)
        for k in range(self.H):
            for inside, vals in pieces:
                if inside(k):
                    rho[k], p[k] = vals[k]
                    break
        # the half cells outside the walls hold the one-sided wall values
        mean = (integral + 0.5 * (down[0][0] + last[self.H - 1][0])) / self.H
        return rho, p, mean, interfaces

    def solve(self, config):
        """The profile whose mean density is <rho>: a dict with rho, p, T at
        the nodes and the interface heights; raises NoSolution."""
        reasons = set()

        def resid(h):
            try:
                return self.profile(config, h)[2] - self.mean
            except NoSolution as e:
                reasons.add(str(e))
                return None

        prev_h, prev_r = None, None
        for k in range(self.H):
            r = resid(float(k))
            if r is not None and r == 0.0:
                return self._result(config, float(k))
            if r is not None and prev_r is not None and (r > 0.0) != (prev_r > 0.0):
                lo, hi, rlo = prev_h, float(k), prev_r
                while hi - lo > 1e-12:
                    mid = 0.5 * (lo + hi)
                    rm = resid(mid)
                    if rm is None:
                        raise NoSolution("the bracket holds a placement that cannot exist")
                    if rm == 0.0:
                        return self._result(config, mid)
                    if (rm > 0.0) == (rlo > 0.0):
                        lo, rlo = mid, rm
                    else:
                        hi = mid
                return self._result(config, 0.5 * (lo + hi))
            prev_h, prev_r = float(k), r
        raise NoSolution(f"no {config} profile holds this mean density"
                         + (" (" + "; ".join(sorted(reasons)) + ")" if reasons else ""))

    def _result(self, config, h):
        rho, p, mean, interfaces = self.profile(config, h)
        T = np.array([self.T(k) for k in range(self.H)])
        return dict(config=config, rho=rho, p=p, T=T, mean=mean, interfaces=interfaces)


def existing_configs(P, H, T_bot, T_top, g, form, mean, m=8, rho_v=0.0):
    """Which of L-V, V-L and V-L-V exist for the column (Sec. VI)."""
    c = Column(P, H, T_bot, T_top, g, form, mean, m, rho_v)
    out = {}
    for cfg in CONFIGS:
        try:
            out[cfg] = c.solve(cfg)
        except NoSolution:
            out[cfg] = None
    return out
