// Host-side FP64 Carnahan-Starling equation of state shared by the C ABI's
// EOS utilities and the sharp-interface column theory.
#pragma once

#include <algorithm>
#include <cmath>

#include "../../include/tplbm.h"

namespace tplbm {
namespace eos {

// ---------------------------------------------------------------------------
// FP64 equation of state.  Carnahan-Starling (Eq. EOS):
//   p = rho R T Z(eta) - a rho^2,  eta = b rho / 4,
//   Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3.
// With h(eta) = eta Z(eta): dp/drho = R T h'(eta) - 2 a rho and
// d2p/drho2 = (b/4) R T h''(eta) - 2 a, where
//   h'  = (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4)/(1 - eta)^4,
//   h'' = (8 + 20 eta - 4 eta^2)/(1 - eta)^5.
// Coexistence (Eq. MaxwellRule) is solved as equal pressure and equal
// chemical potential mu = p/rho + R T [ln eta + (4 eta - 3 eta^2)/(1-eta)^2]
// - a rho (the equal-area rule written as mu_v = mu_l).
// ---------------------------------------------------------------------------
struct CS {
    double a, b, R;
    double Z(double e) const { return (1 + e + e * e - e * e * e) / ((1 - e) * (1 - e) * (1 - e)); }
    double h1(double e) const
    {
        const double s = 1 - e;
        return (1 + 4 * e + 4 * e * e - 4 * e * e * e + e * e * e * e) / (s * s * s * s);
    }
    double h2(double e) const
    {
        const double s = 1 - e;
        return (8 + 20 * e - 4 * e * e) / (s * s * s * s * s);
    }
    double h3(double e) const  // derivative of h2
    {
        const double s = 1 - e;
        return ((20 - 8 * e) * s + 5 * (8 + 20 * e - 4 * e * e)) / (s * s * s * s * s * s);
    }
    double p(double r, double T) const { return r * R * T * Z(b * r / 4) - a * r * r; }
    double dp(double r, double T) const { return R * T * h1(b * r / 4) - 2 * a * r; }
    double d2p(double r, double T) const { return b / 4 * R * T * h2(b * r / 4) - 2 * a; }
    double mu(double r, double T) const
    {
        const double e = b * r / 4;
        return p(r, T) / r + R * T * (std::log(e) + (4 * e - 3 * e * e) / ((1 - e) * (1 - e))) - a * r;
    }
    double rho_max() const { return 4.0 / b; }
};

// root of a monotone function on [lo, hi] by safeguarded Newton
template <class F, class D>
inline double newton_bracket(F f, D df, double lo, double hi, double target, int &ok)
{
    double flo = f(lo) - target, fhi = f(hi) - target;
    ok = (flo <= 0) != (fhi <= 0) || flo == 0 || fhi == 0;
    if (!ok) return 0.5 * (lo + hi);
    const bool inc = fhi > flo;
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double fx = f(x) - target;
        if (fx == 0) return x;
        if ((fx > 0) == inc) hi = x; else lo = x;
        const double d = df(x);
        double xn = (d != 0) ? x - fx / d : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-16 * std::fabs(x) || hi - lo <= 1e-17 * std::fabs(x)) return xn;
        x = xn;
    }
    return x;
}

inline int cs_spinodal(const CS &m, double T, double &sv, double &sl)
{
    int ok;
    const double top = m.rho_max() * (1 - 1e-12);
    // inflection of p(rho): d2p/drho2 = 0, increasing in rho
    const double ri = newton_bracket([&](double r) { return m.d2p(r, T); },
                                     [&](double r) { return m.b * m.b / 16 * m.R * T * m.h3(m.b * r / 4); },
                                     1e-12, top, 0.0, ok);
    if (!ok || m.dp(ri, T) >= 0) return TPLBM_EINVAL;
    sv = newton_bracket([&](double r) { return m.dp(r, T); }, [&](double r) { return m.d2p(r, T); },
                        1e-14, ri, 0.0, ok);
    if (!ok) return TPLBM_ENOTCONVERGED;
    sl = newton_bracket([&](double r) { return m.dp(r, T); }, [&](double r) { return m.d2p(r, T); },
                        ri, top, 0.0, ok);
    if (!ok) return TPLBM_ENOTCONVERGED;
    return TPLBM_OK;
}

// Critical point: rho d2p/drho2 = dp/drho and dp/drho = 0, i.e.
// eta h''(eta) = h'(eta) for the reduced density, then T_c from dp/drho = 0.
inline int cs_critical(const CS &m, double &rc, double &Tc, double &pc)
{
    int ok;
    const double eta = newton_bracket([&](double e) { return e * m.h2(e) - m.h1(e); },
                                      [&](double e) { return e * m.h3(e); }, 1e-3, 0.5, 0.0, ok);
    if (!ok) return TPLBM_ENOTCONVERGED;
    rc = 4 * eta / m.b;
    Tc = 8 * m.a / (m.b * m.R * m.h2(eta));
    pc = m.p(rc, Tc);
    return TPLBM_OK;
}

// Maxwell coexistence at T < T_c: equal pressure and equal chemical potential
// on the two branches (Eq. MaxwellRule).  Bisection on the pressure between
// the spinodal pressures (clipped at zero), Newton roots on each branch.
inline int cs_coexistence(const CS &m, double T, double &rv, double &rl, double &ps)
{
    double sv, sl;
    int rc = cs_spinodal(m, T, sv, sl);
    if (rc) return rc;
    const double top = m.rho_max() * (1 - 1e-13);
    double plo = std::max(m.p(sl, T), 0.0), phi = m.p(sv, T);
    auto branches = [&](double pt, double &v, double &l) {
        int ok1, ok2;
        v = newton_bracket([&](double r) { return m.p(r, T); }, [&](double r) { return m.dp(r, T); },
                           1e-15, sv, pt, ok1);
        l = newton_bracket([&](double r) { return m.p(r, T); }, [&](double r) { return m.dp(r, T); },
                           sl, top, pt, ok2);
        return ok1 && ok2;
    };
    // mu_l - mu_v decreases as the trial pressure rises
    for (int it = 0; it < 400; ++it) {
        const double pt = 0.5 * (plo + phi);
        if (!branches(pt, rv, rl)) return TPLBM_ENOTCONVERGED;
        const double dmu = m.mu(rl, T) - m.mu(rv, T);
        const double plo0 = plo, phi0 = phi;
        if (dmu > 0) plo = pt; else phi = pt;
        if (plo == plo0 && phi == phi0) break;  // the bracket can shrink no further
    }
    ps = 0.5 * (plo + phi);
    if (!branches(ps, rv, rl)) return TPLBM_ENOTCONVERGED;
    return TPLBM_OK;
}

}  // namespace eos
}  // namespace tplbm
