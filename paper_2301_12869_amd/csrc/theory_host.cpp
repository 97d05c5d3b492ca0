// Sharp-interface theoretical equilibrium of a column: the tplbm_theory_*
// calls of include/tplbm.h (Sec. IV A and the appendix on the numerical
// procedure; the L-V, V-L and V-L-V configurations of Sec. VI).
//
// At rest the column obeys dp/dy = F_g,y(rho) (Eq. Momentum_Balance_TS) with
// T linear between the walls (Eq. Temp_Profile).  An interface at height h
// joins the Maxwell coexistence states of T(h) (Eq. MaxwellRule); away from it
// the pressure advances by explicit Euler steps p += F(rho) dy and the density
// is the inverse EOS on the phase's stable or metastable branch
// (Eqs. Inverse_EOS, Numerical_Vapor_Region, Numerical_Liquid_Region).  The
// interface height is searched until the mean density is the requested one.
//
// Discretisation (the paper leaves it open): node intervals split into
// `substeps` equal Euler steps, an interval holding an interface split there;
// a second V-L-V interface placed inside the Euler step where p - p_sat
// changes sign, by linear interpolation; the mean density is the integral of
// the sharp profile over the node cells [-1/2, H - 1/2] (trapezoids over the
// Euler steps plus a half cell at each wall); the interface is tried on every
// node from the bottom up and the first neighbouring pair that brackets the
// mean is bisected to 1e-12.  Columns are independent and solved on host
// threads.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tplbm.h"
#include "eos_host.hpp"

using namespace tplbm::eos;

namespace {

thread_local std::string g_terr = "no error";

int tfail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_terr = buf;
    return code;
}

enum Phase { VAPOUR, LIQUID };

struct Node {
    double rho, p;
};

struct Spinodal {
    double T = std::numeric_limits<double>::quiet_NaN();
    double v = 0, l = 0, pv = 0, pl = 0;
    bool ok = false;
};

struct Coexistence {
    double T = std::numeric_limits<double>::quiet_NaN();
    double v = 0, l = 0, p = 0;
    bool ok = false;
};

// One column.  The spinodal and coexistence solves are cached on the exact
// temperature (a uniform-T column asks for the same one at every step).
class ColumnSolver {
public:
    ColumnSolver(const CS &m, double Tc, const tplbm_theory_column &c)
        : m_(m), Tc_(Tc), c_(c), H_(c.height), below_(c.height), above_(c.height), top_(c.height)
    {
    }

    // Fills rho/p (may be NULL) and res; returns the result status.
    int solve(double *rho, double *p, tplbm_theory_result &res)
    {
        res = tplbm_theory_result{};
        uint32_t seen = 0;
        double mean;
        auto resid = [&](double h, double &r) {
            const uint32_t why = profile(h, nullptr, nullptr, mean, nullptr);
            seen |= why;
            r = mean - c_.mean_rho;
            return why == 0;
        };
        bool have_prev = false;
        double prev_h = 0, prev_r = 0;
        for (int k = 0; k < H_; ++k) {
            double r;
            const bool ok = resid(k, r);
            if (ok && r == 0) return finish(k, rho, p, res);
            if (ok && have_prev && (r > 0) != (prev_r > 0)) {
                double lo = prev_h, hi = k, rlo = prev_r;
                while (hi - lo > 1e-12) {
                    const double mid = 0.5 * (lo + hi);
                    double rm;
                    if (!resid(mid, rm)) return no_solution(seen | TPLBM_THEORY_BROKEN_BRACKET, rho, p, res);
                    if (rm == 0) return finish(mid, rho, p, res);
                    if ((rm > 0) == (rlo > 0)) {
                        lo = mid;
                        rlo = rm;
                    } else {
                        hi = mid;
                    }
                }
                return finish(0.5 * (lo + hi), rho, p, res);
            }
            have_prev = ok;
            prev_h = k;
            prev_r = r;
        }
        return no_solution(seen | TPLBM_THEORY_NO_MATCH, rho, p, res);
    }

private:
    double T(double y) const { return c_.T_bot + (c_.T_top - c_.T_bot) * y / (H_ - 1); }

    // F_g,y of Eqs. Gravity_1 / Gravity_2 / Gravity_3 with y up and g > 0 pointing down
    double F(double rho) const
    {
        if (c_.gravity_form == 2) return -(rho - c_.mean_rho) * c_.g;
        if (c_.gravity_form == 3) return -(rho - c_.rho_v) * c_.g;
        return -rho * c_.g;
    }

    const Spinodal &spinodal(double T)
    {
        if (T != sp_.T) {
            sp_.T = T;
            sp_.ok = cs_spinodal(m_, T, sp_.v, sp_.l) == TPLBM_OK;
            if (sp_.ok) {
                sp_.pv = m_.p(sp_.v, T);
                sp_.pl = m_.p(sp_.l, T);
            }
        }
        return sp_;
    }

    const Coexistence &coexistence(double T)
    {
        if (T != co_.T) {
            co_.T = T;
            co_.ok = cs_coexistence(m_, T, co_.v, co_.l, co_.p) == TPLBM_OK;
        }
        return co_;
    }

    // rho on the phase's branch with p_EOS(rho, T) = p (Eq. Inverse_EOS);
    // above T_c the single branch.  Newton from the neighbour's density,
    // kept inside a shrinking bracket on the monotone branch.
    uint32_t invert(double p, double T, Phase ph, double guess, double &rho)
    {
        double lo, hi;
        if (T >= Tc_) {
            if (!(p > 0)) return TPLBM_THEORY_ZERO_PRESSURE;
            lo = 0;
            hi = m_.rho_max();
        } else {
            const Spinodal &s = spinodal(T);
            if (!s.ok) return TPLBM_THEORY_SOLVE_FAILED;
            if (ph == VAPOUR) {
                if (!(p > 0)) return TPLBM_THEORY_ZERO_PRESSURE;
                if (p > s.pv) return TPLBM_THEORY_NO_VAPOUR;
                lo = 0;
                hi = s.v;
            } else {
                if (p < s.pl) return TPLBM_THEORY_NO_LIQUID;
                lo = s.l;
                hi = m_.rho_max();
            }
        }
        double x = (guess > lo && guess < hi) ? guess : 0.5 * (lo + hi);
        for (int it = 0; it < 200; ++it) {
            const double f = m_.p(x, T) - p;
            if (f == 0) break;
            (f > 0 ? hi : lo) = x;
            const double d = m_.dp(x, T);
            double xn = d > 0 ? x - f / d : 0.5 * (lo + hi);
            if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
            const bool done = std::fabs(xn - x) <= 1e-15 * x || hi - lo <= 1e-15 * hi;
            x = xn;
            if (done) break;
        }
        rho = x;
        return 0;
    }

    // Euler march from (y0, p0, rho0) to the top (up) or bottom wall, storing
    // the nodes it reaches (a node at y0 itself included) in `out` and the
    // trapezoidal integral of rho over its span.  With `watch`, stops where
    // p - p_sat(T) changes sign and reports that point in (ys, ps).
    uint32_t march(double y0, double p0, double rho0, Phase ph, bool up, bool watch, std::vector<Node> &out,
                   double &integral, bool &switched, double &ys, double &ps)
    {
        integral = 0;
        switched = false;
        double y = y0, p = p0, rho = rho0, d_prev = 0;
        if (watch && T(y) < Tc_) {
            const Coexistence &cx = coexistence(T(y));
            if (!cx.ok) return TPLBM_THEORY_SOLVE_FAILED;
            d_prev = p - cx.p;
        }
        const int dir = up ? 1 : -1;
        const int last = up ? H_ - 1 : 0;
        for (int node = up ? (int)std::ceil(y0) : (int)std::floor(y0); up ? node <= last : node >= last;
             node += dir) {
            const double step = (node - y) / c_.substeps;
            if (step != 0) {
                for (int s = 0; s < c_.substeps; ++s) {
                    const double p_new = p + F(rho) * step;
                    const double y_new = y + step;
                    if (watch && T(y_new) < Tc_) {
                        const Coexistence &cx = coexistence(T(y_new));
                        if (!cx.ok) return TPLBM_THEORY_SOLVE_FAILED;
                        const double d_new = p_new - cx.p;
                        if (d_prev != 0 && (d_new == 0 || (d_new > 0) != (d_prev > 0))) {
                            const double f = d_prev / (d_prev - d_new);
                            ys = y + f * step;
                            ps = p + f * (p_new - p);
                            double rs;
                            if (uint32_t why = invert(ps, T(ys), ph, rho, rs)) return why;
                            integral += 0.5 * (rho + rs) * std::fabs(ys - y);
                            switched = true;
                            return 0;
                        }
                        d_prev = d_new;
                    }
                    double rho_new;
                    if (uint32_t why = invert(p_new, T(y_new), ph, rho, rho_new)) return why;
                    integral += 0.5 * (rho + rho_new) * std::fabs(step);
                    y = y_new;
                    p = p_new;
                    rho = rho_new;
                }
            }
            y = node;
            out[node] = Node{rho, p};
        }
        return 0;
    }

    // The configuration with its (lower) interface at h: node values into
    // rho/p when given, the profile's mean, and the second interface (V-L-V).
    uint32_t profile(double h, double *rho, double *p, double &mean, double *h2)
    {
        const double Ti = T(h);
        if (Ti >= Tc_) return TPLBM_THEORY_SUPERCRITICAL_INTERFACE;
        const Coexistence &cx = coexistence(Ti);
        if (!cx.ok) return TPLBM_THEORY_SOLVE_FAILED;
        const double rv = cx.v, rl = cx.l, psat = cx.p;
        const bool lv = c_.config == TPLBM_THEORY_LV, vlv = c_.config == TPLBM_THEORY_VLV;
        double i_down, i_up, i_top = 0, y2 = 0, p2 = 0, unused;
        bool sw;
        if (uint32_t why = march(h, psat, lv ? rl : rv, lv ? LIQUID : VAPOUR, false, false, below_, i_down, sw,
                                 unused, unused))
            return why;
        if (uint32_t why = march(h, psat, lv ? rv : rl, lv ? VAPOUR : LIQUID, true, vlv, above_, i_up, sw, y2, p2))
            return why;
        if (vlv) {
            if (!sw) return TPLBM_THEORY_NO_SECOND_INTERFACE;
            const Coexistence &c2 = coexistence(T(y2));
            if (!c2.ok) return TPLBM_THEORY_SOLVE_FAILED;
            const double rv2 = c2.v, ps2 = c2.p;
            if (uint32_t why = march(y2, ps2, rv2, VAPOUR, true, false, top_, i_top, sw, unused, unused))
                return why;
        }
        const std::vector<Node> &upper_wall = vlv ? top_ : above_;
        mean = (i_down + i_up + i_top + 0.5 * (below_[0].rho + upper_wall[H_ - 1].rho)) / H_;
        if (h2) *h2 = y2;
        if (rho || p) {
            for (int k = 0; k < H_; ++k) {
                const Node &n = k <= h ? below_[k] : (!vlv || k < y2) ? above_[k] : top_[k];
                if (rho) rho[k] = n.rho;
                if (p) p[k] = n.p;
            }
        }
        return 0;
    }

    int finish(double h, double *rho, double *p, tplbm_theory_result &res)
    {
        double mean, h2 = 0;
        if (uint32_t why = profile(h, rho, p, mean, &h2)) return no_solution(why, rho, p, res);
        res.status = TPLBM_OK;
        res.n_interfaces = c_.config == TPLBM_THEORY_VLV ? 2 : 1;
        res.interface[0] = h;
        res.interface[1] = c_.config == TPLBM_THEORY_VLV ? h2 : std::numeric_limits<double>::quiet_NaN();
        res.mean_rho = mean;
        return TPLBM_OK;
    }

    int no_solution(uint32_t reasons, double *rho, double *p, tplbm_theory_result &res)
    {
        const double nan = std::numeric_limits<double>::quiet_NaN();
        for (int k = 0; k < H_; ++k) {
            if (rho) rho[k] = nan;
            if (p) p[k] = nan;
        }
        res.status = TPLBM_ENOSOLUTION;
        res.reasons = reasons;
        res.interface[0] = res.interface[1] = res.mean_rho = nan;
        return TPLBM_ENOSOLUTION;
    }

    const CS &m_;
    const double Tc_;
    const tplbm_theory_column c_;
    const int H_;
    std::vector<Node> below_, above_, top_;
    Spinodal sp_;
    Coexistence co_;
};

}  // namespace

extern "C" int tplbm_theory_solve(double a, double b, double R, int32_t ncols, const tplbm_theory_column *cols,
                                  double *rho, double *p, tplbm_theory_result *out, int32_t nthreads)
{
    if (!(a > 0 && b > 0 && R > 0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(R))
        return tfail(TPLBM_EINVAL, "need finite a, b, R > 0");
    if (ncols < 0 || (ncols > 0 && (!cols || !out))) return tfail(TPLBM_EINVAL, "need ncols >= 0, columns and results");
    const CS m{a, b, R};
    double rc, Tc, pc;
    if (cs_critical(m, rc, Tc, pc)) return tfail(TPLBM_ENOTCONVERGED, "critical point not bracketed");
    std::vector<int64_t> off(ncols + 1, 0);
    for (int32_t i = 0; i < ncols; ++i) {
        const tplbm_theory_column &c = cols[i];
        if (c.height < 3 || c.height > (1 << 24)) return tfail(TPLBM_ESHAPE, "column %d: height %d outside 3 .. 2^24", i, c.height);
        if (c.gravity_form < 1 || c.gravity_form > 3) return tfail(TPLBM_EINVAL, "column %d: gravity form must be 1, 2 or 3", i);
        if (!std::isfinite(c.rho_v)) return tfail(TPLBM_EINVAL, "column %d: rho_v must be finite", i);
        if (c.config < TPLBM_THEORY_LV || c.config > TPLBM_THEORY_VLV) return tfail(TPLBM_EINVAL, "column %d: unknown configuration", i);
        if (c.substeps < 1 || c.substeps > 4096) return tfail(TPLBM_EINVAL, "column %d: substeps outside 1 .. 4096", i);
        if (!(c.T_bot > 0 && c.T_top > 0) || !std::isfinite(c.T_bot) || !std::isfinite(c.T_top))
            return tfail(TPLBM_EINVAL, "column %d: wall temperatures must be finite and > 0", i);
        if (!std::isfinite(c.g)) return tfail(TPLBM_EINVAL, "column %d: g must be finite", i);
        if (!(c.mean_rho > 0 && c.mean_rho < m.rho_max()))
            return tfail(TPLBM_EINVAL, "column %d: mean density must lie in (0, 4/b)", i);
        off[i + 1] = off[i] + c.height;
    }
    if (ncols > 0 && !rho) return tfail(TPLBM_EINVAL, "rho is NULL");
    int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
    nt = std::max(1, std::min(nt, (int)ncols));
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (int32_t i; (i = next.fetch_add(1)) < ncols;) {
            ColumnSolver s(m, Tc, cols[i]);
            s.solve(rho + off[i], p ? p + off[i] : nullptr, out[i]);
        }
    };
    if (nt == 1) {
        work();
    } else {
        std::vector<std::thread> pool;
        try {
            for (int t = 0; t < nt; ++t) pool.emplace_back(work);
        } catch (...) {
            // fewer threads than asked for: the ones started and this one finish the work
        }
        work();
        for (auto &t : pool) t.join();
    }
    return TPLBM_OK;
}

extern "C" const char *tplbm_theory_last_error(void) { return g_terr.c_str(); }
