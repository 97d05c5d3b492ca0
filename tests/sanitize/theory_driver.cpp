// Host-only driver for the sanitizer builds of the sharp-interface theory
// solver (tplbm_theory_solve): a mixed batch of columns -- every
// configuration and gravity form, both gravity signs, heating from above and
// below, columns without a solution -- solved on 1, 4 and an automatic
// number of threads, whose results must agree bit for bit; then the
// rejection of a bad column.  Exits 0 on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tplbm.h"

namespace {

// Carnahan-Starling constants of the paper's runs and, to seven digits, the
// critical point they give (b rho_c = 0.5217755, b R T_c / a = 0.3773148);
// the columns only need to fall on both sides of the existence limits
constexpr double kA = 0.5, kB = 4.0, kR = 1.0;
constexpr double kTc = 0.3773148 * kA / (kB * kR);
constexpr double kRhoC = 0.5217755 / kB;

std::vector<tplbm_theory_column> columns()
{
    std::vector<tplbm_theory_column> c;
    const double mean = 1.3344 * kRhoC;
    const int cfgs[3] = {TPLBM_THEORY_LV, TPLBM_THEORY_VL, TPLBM_THEORY_VLV};
    int k = 0;
    for (int form = 1; form <= 3; ++form)
        for (int cfg : cfgs)
            for (double g : {2e-5, -2e-5, 6e-5})
                for (double dt : {0.2, -0.1, 0.0}) {
                    tplbm_theory_column col{};
                    col.height = 31 + 7 * (k++ % 5);
                    col.gravity_form = form;
                    col.config = cfg;
                    col.substeps = 2;
                    col.T_bot = (0.75 + dt / 2) * kTc;
                    col.T_top = (0.75 - dt / 2) * kTc;
                    col.g = g;
                    col.mean_rho = mean;
                    col.rho_v = form == 3 ? 0.12 * kRhoC : 0.0;
                    c.push_back(col);
                }
    return c;
}

struct Out {
    std::vector<double> rho, p;
    std::vector<tplbm_theory_result> res;
};

int solve(const std::vector<tplbm_theory_column> &c, int threads, Out &o)
{
    size_t n = 0;
    for (const auto &col : c) n += (size_t)col.height;
    o.rho.assign(n, 0.0);
    o.p.assign(n, 0.0);
    o.res.assign(c.size(), tplbm_theory_result{});
    return tplbm_theory_solve(kA, kB, kR, (int32_t)c.size(), c.data(), o.rho.data(), o.p.data(), o.res.data(),
                              threads);
}

bool same_bits(const std::vector<double> &a, const std::vector<double> &b)
{
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(double)) == 0;
}

}  // namespace

int main()
{
    const auto c = columns();
    Out one, four, any;
    if (solve(c, 1, one) != TPLBM_OK || solve(c, 4, four) != TPLBM_OK || solve(c, 0, any) != TPLBM_OK) {
        std::fprintf(stderr, "solve failed: %s\n", tplbm_theory_last_error());
        return 1;
    }
    int found = 0;
    for (size_t k = 0; k < c.size(); ++k) found += one.res[k].status == TPLBM_OK;
    if (found == 0 || found == (int)c.size()) {
        std::fprintf(stderr, "expected a mix of columns with and without a solution, got %d of %zu\n", found,
                     c.size());
        return 1;
    }
    for (const Out *o : {&four, &any}) {
        if (!same_bits(one.rho, o->rho) || !same_bits(one.p, o->p) ||
            std::memcmp(one.res.data(), o->res.data(), one.res.size() * sizeof(tplbm_theory_result)) != 0) {
            std::fprintf(stderr, "results depend on the thread count\n");
            return 1;
        }
    }
    // a bad column: rejected, nothing written, a message kept
    auto bad = c;
    bad[3].height = 2;
    Out b;
    const int rc = solve(bad, 4, b);
    if (rc == TPLBM_OK || std::strlen(tplbm_theory_last_error()) == 0) {
        std::fprintf(stderr, "a bad column was not rejected\n");
        return 1;
    }
    std::printf("theory driver: %zu columns, %d with a solution, identical on 1, 4 and all threads\n", c.size(),
                found);
    return 0;
}
