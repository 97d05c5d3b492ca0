/*
 * tplbm_oracle.c -- plain FP64 CPU oracle of the thermal pseudopotential
 * lattice Boltzmann update of Czelusniak, Cabezas Gomez and Wagner,
 * "Effects of gravity induced pressure variations for thermal liquid-gas
 * phase-change simulations with the pseudopotential lattice Boltzmann method"
 * (arXiv 2301.12869).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark load
 * it.  It shares no code, header, table or constant generator with the GPU
 * library, and neither side includes or links the other.
 *
 * Style: plain loops over nodes in index order, FP64 throughout, every
 * intermediate field materialised, no fusion, no blocking.  Built with
 * -ffp-contract=off so that every product and sum is rounded as written.
 *
 * Layouts (structure of arrays, x fastest):
 *   D2Q9 : f[i*N + y*nx + x],            N = nx*ny,   wall-normal axis y
 *   D1Q3 : f[i*ny + y],                  wall-normal axis y (one column)
 *   D3Q19: f[i*N + (z*ny + y)*nx + x],   N = nx*ny*nz, wall-normal axis z
 * The state held between steps is f^n: the populations at time n, after
 * streaming and after the wall reconstruction.  T holds T^n.  Wall nodes
 * (first and last layer along the wall-normal axis, when walls are on) keep
 * the temperature they were given (Dirichlet).
 *
 * Readings of points the paper leaves open (see the design notes):
 *   - G = -1, c = 1 in the pseudopotential (the sign that makes the square
 *     root real for the Carnahan-Starling EOS at lattice parameters).
 *   - At wall nodes the total force is zero (interaction and gravity), so
 *     the wall collision is force free.
 *   - <rho> is the mean over all nodes, wall nodes included, of rho^n.
 *   - Temperature: Heun's two-stage Runge-Kutta with rho and u frozen at n.
 *   - The steady test uses max |u^n| over all nodes.
 * Parity unpinned: the transient between the pinned limits (nucleation
 * times, metastable life times) is checked only against the GPU path.
 *
 * Threads: orc_set_threads(n) lets the D2Q9 and D3Q19 node loops run on n
 * OpenMP threads (default 1, the plain definition).  Every node's arithmetic
 * is the same on any thread, each output is written by one iteration, the
 * flags are OR-ed (order-free), and the sums (mass, <rho>) stay serial in
 * index order, so the results are bit for bit those of one thread.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int orc_threads = 1;

/* number of threads for the node loops (>= 1); returns the previous value */
int orc_set_threads(int n)
{
    int prev = orc_threads;
    orc_threads = n < 1 ? 1 : n;
    return prev;
}

typedef struct {
    int32_t lattice;      /* 1: D1Q3 column, 2: D2Q9, 3: D3Q19 */
    int32_t nx, ny, nz;   /* D1Q3 uses ny only; D2Q9 nx, ny; D3Q19 all */
    int32_t walls;        /* 1: wet-node walls at both ends of the wall-normal axis; 0: periodic */
    int32_t eos;          /* 0: Carnahan-Starling; 1: ideal lattice gas p = rho/3 (psi = 0) */
    int32_t gravity_form; /* 1: F = rho g; 2: F = (rho - <rho>) g; 3: F = (rho - rho_v) g */
    int32_t pad0;
    double a, b, R, G, sigma;
    double tau[6];        /* tau_rho, tau_e, tau_varsigma, tau_j, tau_q, tau_nu */
    double cv, kappa;
    double g;             /* gravity magnitude; g > 0 points down the wall-normal axis */
    double rho_v;         /* form 3: the vapour density of Eq. Gravity_3 */
} orc_params;

/* gravity along the wall-normal axis (Eqs. Gravity_1, Gravity_2, Gravity_3):
 * F = -(rho - s) g with s = 0, <rho> or rho_v */
static double gravity(const orc_params *P, double rho, double mean)
{
    if (P->gravity_form == 2) return -(rho - mean) * P->g;
    if (P->gravity_form == 3) return -(rho - P->rho_v) * P->g;
    return -rho * P->g;
}

/* status / flags */
#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EUNSUPPORTED 3
#define ORC_FLAG_NAN 1
#define ORC_FLAG_RHO 2
#define ORC_FLAG_ETA 4
#define ORC_FLAG_PSI 8

/* diagnostics written by a step call: values of the last step's time level n */
typedef struct {
    double mass;      /* sum of rho^n over all nodes */
    double mean_rho;  /* <rho>^n */
    double max_u;     /* max |u^n| */
    double min_rho;   /* min rho^n */
    double flags;     /* OR of ORC_FLAG_* seen during the call (as a double) */
} orc_diag;

/* ======================================================================
 * Equation of state (Carnahan-Starling, the paper's Eq. EOS in Sec. IV.B)
 * ====================================================================== */

/* compressibility factor of the Carnahan-Starling EOS, eta = b rho / 4 */
static double cs_factor(double eta)
{
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    return num / den;
}

double orc_eos_p(const orc_params *P, double rho, double T)
{
    if (P->eos == 1)
        return rho / 3.0;
    double eta = P->b * rho / 4.0;
    return rho * P->R * T * cs_factor(eta) - P->a * rho * rho;
}

/* (dp/dT) at constant rho, used by the energy equation (Eq. Energy_Equation) */
double orc_eos_dpdT(const orc_params *P, double rho, double T)
{
    (void)T;
    if (P->eos == 1)
        return 0.0;
    double eta = P->b * rho / 4.0;
    return rho * P->R * cs_factor(eta);
}

/* d(eta Z)/d eta and its derivative, closed forms of the C-S hard-sphere term */
static double cs_g1(double eta)
{
    double num = 1.0 + 4.0 * eta + 4.0 * eta * eta - 4.0 * eta * eta * eta + eta * eta * eta * eta;
    double s = 1.0 - eta;
    return num / (s * s * s * s);
}
static double cs_g2(double eta)
{
    double s = 1.0 - eta;
    return 4.0 * (2.0 + 5.0 * eta - eta * eta) / (s * s * s * s * s);
}

/* (dp/drho)_T */
double orc_eos_dpdrho(const orc_params *P, double rho, double T)
{
    if (P->eos == 1)
        return 1.0 / 3.0;
    double eta = P->b * rho / 4.0;
    return P->R * T * cs_g1(eta) - 2.0 * P->a * rho;
}

/* (d2p/drho2)_T */
double orc_eos_d2pdrho2(const orc_params *P, double rho, double T)
{
    if (P->eos == 1)
        return 0.0;
    double eta = P->b * rho / 4.0;
    return P->R * T * cs_g2(eta) * P->b / 4.0 - 2.0 * P->a;
}

/* Critical point: dp/drho = d2p/drho2 = 0.  Eliminating T gives
 * eta g2(eta) = g1(eta); solved by bisection, then T_c from d2p/drho2 = 0. */
int orc_critical(double a, double b, double R, double *out3)
{
    double lo = 1e-3, hi = 0.5;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        double h = mid * cs_g2(mid) - cs_g1(mid);
        double hlo = lo * cs_g2(lo) - cs_g1(lo);
        if ((h < 0) == (hlo < 0))
            lo = mid;
        else
            hi = mid;
    }
    double eta_c = 0.5 * (lo + hi);
    double rho_c = 4.0 * eta_c / b;
    double T_c = 2.0 * a / (R * cs_g2(eta_c) * b / 4.0);
    orc_params P;
    memset(&P, 0, sizeof P);
    P.a = a; P.b = b; P.R = R; P.eos = 0;
    out3[0] = rho_c;
    out3[1] = T_c;
    out3[2] = orc_eos_p(&P, rho_c, T_c);
    return ORC_OK;
}

/* Spinodal densities at temperature T (local extrema of p(rho), Sec. V).
 * out2 = {rho_spinodal_vapour, rho_spinodal_liquid}.  EINVAL above T_c. */
int orc_spinodal(const orc_params *P, double T, double *out2)
{
    /* d2p/drho2 increases with rho: its root splits the two extrema */
    double lo = 1e-12, hi = 4.0 / P->b * (1.0 - 1e-9);
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_eos_d2pdrho2(P, mid, T) < 0)
            lo = mid;
        else
            hi = mid;
    }
    double rho_m = 0.5 * (lo + hi);
    if (orc_eos_dpdrho(P, rho_m, T) >= 0)
        return ORC_EINVAL; /* no van der Waals loop: supercritical */
    double a = 1e-12, c = rho_m;
    for (int it = 0; it < 200; ++it) { /* dp/drho > 0 below the vapour spinodal */
        double mid = 0.5 * (a + c);
        if (orc_eos_dpdrho(P, mid, T) > 0) a = mid; else c = mid;
    }
    out2[0] = 0.5 * (a + c);
    a = rho_m; c = 4.0 / P->b * (1.0 - 1e-9);
    for (int it = 0; it < 200; ++it) { /* dp/drho > 0 above the liquid spinodal */
        double mid = 0.5 * (a + c);
        if (orc_eos_dpdrho(P, mid, T) < 0) a = mid; else c = mid;
    }
    out2[1] = 0.5 * (a + c);
    return ORC_OK;
}

/* Antiderivative of p/rho^2 in rho for Carnahan-Starling:
 *   int p/rho^2 drho = R T [ ln eta + (4 eta - 3 eta^2)/(1-eta)^2 ] - a rho  (+const)
 * (the C-S hard-sphere free energy).  Used by the equal-area rule. */
static double cs_int_p_over_rho2(const orc_params *P, double rho, double T)
{
    double eta = P->b * rho / 4.0;
    double s = 1.0 - eta;
    return P->R * T * (log(eta) + (4.0 * eta - 3.0 * eta * eta) / (s * s)) - P->a * rho;
}

/* density on one monotone branch where p(rho) = p_target, by bisection */
static double branch_root(const orc_params *P, double T, double p_target, double lo, double hi)
{
    /* p is increasing on [lo, hi] */
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi), lo0 = lo, hi0 = hi;
        if (orc_eos_p(P, mid, T) < p_target) lo = mid; else hi = mid;
        if (lo == lo0 && hi == hi0) break; /* the bracket can shrink no further */
    }
    return 0.5 * (lo + hi);
}

/* Maxwell equal-area rule (Eq. MaxwellRule): p(rho_v) = p(rho_l) = p_sat and
 * int_{rho_v}^{rho_l} (p_sat - p) drho / rho^2 = 0.
 * out3 = {rho_v, rho_l, p_sat}.  EINVAL at or above T_c. */
int orc_coexistence(const orc_params *P, double T, double *out3)
{
    double sp[2];
    if (orc_spinodal(P, T, sp) != ORC_OK)
        return ORC_EINVAL;
    double p_hi = orc_eos_p(P, sp[0], T); /* local maximum (vapour spinodal) */
    double p_lo = orc_eos_p(P, sp[1], T); /* local minimum (liquid spinodal) */
    if (p_lo < 0) p_lo = 0;
    double rho_top = 4.0 / P->b * (1.0 - 1e-12);
    double lo = p_lo, hi = p_hi;
    double rv = 0, rl = 0;
    for (int it = 0; it < 300; ++it) {
        double ps = 0.5 * (lo + hi);
        rv = branch_root(P, T, ps, 1e-14, sp[0]);
        rl = branch_root(P, T, ps, sp[1], rho_top);
        double area = ps * (1.0 / rv - 1.0 / rl)
                      - (cs_int_p_over_rho2(P, rl, T) - cs_int_p_over_rho2(P, rv, T));
        /* area grows with ps; zero area is the coexistence pressure */
        double lo0 = lo, hi0 = hi;
        if (area > 0) hi = ps; else lo = ps;
        if (lo == lo0 && hi == hi0) break;
    }
    double ps = 0.5 * (lo + hi);
    out3[0] = branch_root(P, T, ps, 1e-14, sp[0]);
    out3[1] = branch_root(P, T, ps, sp[1], rho_top);
    out3[2] = ps;
    return ORC_OK;
}

/* pseudopotential (Eq. InteractionPotential) with c = 1, c_s^2 = 1/3 */
static double psi_of(const orc_params *P, double rho, double T, int *flags)
{
    double arg = 2.0 * (orc_eos_p(P, rho, T) - rho / 3.0) / P->G;
    if (P->eos == 0 && P->b * rho / 4.0 >= 1.0)
        *flags |= ORC_FLAG_ETA;
    if (arg < 0) {
        *flags |= ORC_FLAG_PSI;
        return NAN;
    }
    return sqrt(arg);
}

/* ======================================================================
 * D2Q9 (Sec. III): velocity set, weights, MRT matrix
 * ====================================================================== */
static const int C2X[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int C2Y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* Gram-Schmidt moment matrix (Eq. MatrixMRT) */
static const double M2[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* M^{-1}: the rows of M are orthogonal, so M^{-1} = M^T diag(1/|row_k|^2).
 * The row norms are computed here from M itself. */
static void m2_inverse(double Minv[9][9])
{
    double nrm[9];
    for (int k = 0; k < 9; ++k) {
        nrm[k] = 0;
        for (int i = 0; i < 9; ++i) nrm[k] += M2[k][i] * M2[k][i];
    }
    for (int i = 0; i < 9; ++i)
        for (int k = 0; k < 9; ++k) Minv[i][k] = M2[k][i] / nrm[k];
}

/* exported for the algebra tests */
void orc_d2q9_minv(double *out81)
{
    double Mi[9][9];
    m2_inverse(Mi);
    for (int i = 0; i < 9; ++i)
        for (int k = 0; k < 9; ++k) out81[i * 9 + k] = Mi[i][k];
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Li's forcing source (Eq. LiFS): the vector S with
 * (I - Lambda/2)^{-1} M F' = S */
static void d2q9_source(const orc_params *P, double ux, double uy, double Fx, double Fy,
                        double Xp, double S[9])
{
    double uF = ux * Fx + uy * Fy;
    S[0] = 0;
    S[1] = 6.0 * uF + P->sigma * Xp / (P->tau[1] - 0.5);
    S[2] = -6.0 * uF - P->sigma * Xp / (P->tau[2] - 0.5);
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (ux * Fx - uy * Fy);
    S[8] = ux * Fy + uy * Fx;
}

/* Second order equilibrium with the force-corrected velocity
 * (Eq. EquilibriumDistribution), c_s^2 = 1/3. */
static double feq_d2q9(int i, double rho, double ux, double uy)
{
    double cu = C2X[i] * ux + C2Y[i] * uy;
    double uu = ux * ux + uy * uy;
    double cs2 = 1.0 / 3.0;
    double second = 0.0;
    /* (c_a c_b - cs2 delta_ab) rho u_a u_b / (2 cs2^2) */
    second = (cu * cu - cs2 * uu) / (2.0 * cs2 * cs2);
    return W2[i] * (rho + cu / cs2 * rho + second * rho);
}

/* relaxation rates in the moment order of Eq. RelaxationMatrix */
static void d2q9_lambda(const orc_params *P, double L[9])
{
    L[0] = 1.0 / P->tau[0];
    L[1] = 1.0 / P->tau[1];
    L[2] = 1.0 / P->tau[2];
    L[3] = 1.0 / P->tau[3];
    L[4] = 1.0 / P->tau[4];
    L[5] = 1.0 / P->tau[3];
    L[6] = 1.0 / P->tau[4];
    L[7] = 1.0 / P->tau[5];
    L[8] = 1.0 / P->tau[5];
}

/* Shan-Chen nearest-neighbour weights w(|c|^2): w(1) = 1/3, w(2) = 1/12 */
static double wsc2(int i)
{
    int c2 = C2X[i] * C2X[i] + C2Y[i] * C2Y[i];
    if (c2 == 1) return 1.0 / 3.0;
    if (c2 == 2) return 1.0 / 12.0;
    return 0.0;
}

/* Work arrays for one D2Q9 step */
typedef struct {
    double *rho, *psi, *ux, *uy, *Fx, *Fy, *Fix, *Fiy, *Tt, *Tn, *k1, *fs;
} d2_work;

/* The macroscopic fields of time n: rho, psi, forces, u.  Returns <rho>. */
static double d2q9_macro(const orc_params *P, const double *f, const double *T, d2_work *w,
                         int *flags)
{
    int nx = P->nx, ny = P->ny, N = nx * ny;
    int fl = 0;
    /* density (Eq. Density) */
#pragma omp parallel for num_threads(orc_threads) reduction(| : fl)
    for (int n = 0; n < N; ++n) {
        double s = 0;
        for (int i = 0; i < 9; ++i) s += f[i * N + n];
        w->rho[n] = s;
        if (!(s == s)) fl |= ORC_FLAG_NAN;
        if (s <= 0) fl |= ORC_FLAG_RHO;
    }
    /* mean density over all nodes, in index order */
    double tot = 0;
    for (int n = 0; n < N; ++n) tot += w->rho[n];
    double mean = tot / N;
    /* pseudopotential */
#pragma omp parallel for num_threads(orc_threads) reduction(| : fl)
    for (int n = 0; n < N; ++n) w->psi[n] = psi_of(P, w->rho[n], T[n], &fl);
    *flags |= fl;
    /* forces: Shan-Chen (Eq. ShanChenForce) plus gravity (Eqs. Gravity_1/2) */
#pragma omp parallel for num_threads(orc_threads)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int n = y * nx + x;
            int wall = P->walls && (y == 0 || y == ny - 1);
            if (wall) {
                w->Fix[n] = w->Fiy[n] = 0;
                w->Fx[n] = w->Fy[n] = 0;
                continue;
            }
            double sx = 0, sy = 0;
            for (int i = 1; i < 9; ++i) {
                int xx = wrap(x + C2X[i], nx), yy = wrap(y + C2Y[i], ny);
                double ps = w->psi[yy * nx + xx];
                sx += wsc2(i) * ps * C2X[i];
                sy += wsc2(i) * ps * C2Y[i];
            }
            w->Fix[n] = -P->G * w->psi[n] * sx;
            w->Fiy[n] = -P->G * w->psi[n] * sy;
            double fg = gravity(P, w->rho[n], mean);
            w->Fx[n] = w->Fix[n];
            w->Fy[n] = w->Fiy[n] + fg;
        }
    /* force-corrected velocity (Eq. Momentum) */
#pragma omp parallel for num_threads(orc_threads)
    for (int n = 0; n < N; ++n) {
        double jx = 0, jy = 0;
        for (int i = 0; i < 9; ++i) {
            jx += f[i * N + n] * C2X[i];
            jy += f[i * N + n] * C2Y[i];
        }
        w->ux[n] = (jx + w->Fx[n] / 2.0) / w->rho[n];
        w->uy[n] = (jy + w->Fy[n] / 2.0) / w->rho[n];
    }
    return mean;
}

/* Right-hand side of the energy equation (Eq. Energy_Equation) at one
 * interior node, isotropic second-order differences on the D2Q9 stencil. */
static double d2q9_energy_rhs(const orc_params *P, const double *Tf, const d2_work *w, int x,
                              int y)
{
    int nx = P->nx, ny = P->ny, n = y * nx + x;
    double gx = 0, gy = 0, lap = 0, div = 0;
    for (int i = 0; i < 9; ++i) {
        int m = wrap(y + C2Y[i], ny) * nx + wrap(x + C2X[i], nx);
        gx += W2[i] * C2X[i] * Tf[m];
        gy += W2[i] * C2Y[i] * Tf[m];
        lap += W2[i] * (Tf[m] - Tf[n]);
        div += W2[i] * (C2X[i] * w->ux[m] + C2Y[i] * w->uy[m]);
    }
    gx *= 3.0; gy *= 3.0; lap *= 6.0; div *= 3.0;
    double rho = w->rho[n];
    double adv = -(w->ux[n] * gx + w->uy[n] * gy);
    double cond = P->kappa / (rho * P->cv) * lap;
    double work = -Tf[n] / (rho * P->cv) * orc_eos_dpdT(P, rho, Tf[n]) * div;
    return adv + cond + work;
}

static void d2q9_step_once(const orc_params *P, double *f, double *T, d2_work *w, int *flags,
                           orc_diag *dg)
{
    int nx = P->nx, ny = P->ny, N = nx * ny;
    double mean = d2q9_macro(P, f, T, w, flags);

    /* diagnostics of time level n */
    double mass = 0, umax = 0, rmin = INFINITY;
    for (int n = 0; n < N; ++n) {
        mass += w->rho[n];
        double um = sqrt(w->ux[n] * w->ux[n] + w->uy[n] * w->uy[n]);
        if (um > umax) umax = um;
        if (w->rho[n] < rmin) rmin = w->rho[n];
    }
    dg->mass = mass; dg->mean_rho = mean; dg->max_u = umax; dg->min_rho = rmin;

    /* temperature: Heun with rho, u frozen; Dirichlet at the walls */
#pragma omp parallel for num_threads(orc_threads)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int n = y * nx + x;
            int wall = P->walls && (y == 0 || y == ny - 1);
            if (wall) { w->k1[n] = 0; w->Tt[n] = T[n]; continue; }
            w->k1[n] = d2q9_energy_rhs(P, T, w, x, y);
            w->Tt[n] = T[n] + w->k1[n];
        }
#pragma omp parallel for num_threads(orc_threads)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int n = y * nx + x;
            int wall = P->walls && (y == 0 || y == ny - 1);
            if (wall) { w->Tn[n] = T[n]; continue; }
            double k2 = d2q9_energy_rhs(P, w->Tt, w, x, y);
            w->Tn[n] = T[n] + 0.5 * (w->k1[n] + k2);
        }

    /* MRT collision with Li's forcing (Eqs. LBE, OperatorMRT, LiFS) */
    double L[9], nrm[9];
    d2q9_lambda(P, L);
    for (int k = 0; k < 9; ++k) {
        nrm[k] = 0;
        for (int i = 0; i < 9; ++i) nrm[k] += M2[k][i] * M2[k][i];
    }
#pragma omp parallel for num_threads(orc_threads)
    for (int n = 0; n < N; ++n) {
        double fl[9], fe[9], m[9], me[9], S[9], ms[9];
        for (int i = 0; i < 9; ++i) fl[i] = f[i * N + n];
        for (int i = 0; i < 9; ++i) fe[i] = feq_d2q9(i, w->rho[n], w->ux[n], w->uy[n]);
        double Fi2 = w->Fix[n] * w->Fix[n] + w->Fiy[n] * w->Fiy[n];
        double Xp = (Fi2 > 0) ? Fi2 / (w->psi[n] * w->psi[n]) : 0.0;
        d2q9_source(P, w->ux[n], w->uy[n], w->Fx[n], w->Fy[n], Xp, S);
        for (int k = 0; k < 9; ++k) {
            m[k] = 0; me[k] = 0;
            for (int i = 0; i < 9; ++i) { m[k] += M2[k][i] * fl[i]; me[k] += M2[k][i] * fe[i]; }
        }
        /* the mass moment is a collision invariant (Sec. III, after Eq.
         * RelaxationMatrix): its equilibrium value is the density itself */
        me[0] = m[0];
        for (int k = 0; k < 9; ++k)
            ms[k] = m[k] - L[k] * (m[k] - me[k]) + (1.0 - L[k] / 2.0) * S[k];
        /* f* = M^{-1} m* = M^T diag(1/|row_k|^2) m*, dividing by the row norms */
        for (int i = 0; i < 9; ++i) {
            double s = 0;
            for (int k = 0; k < 9; ++k) s += M2[k][i] * (ms[k] / nrm[k]);
            w->fs[i * N + n] = s;
        }
    }

    /* streaming (Eq. LBE): periodic in x; in y periodic or cut at the walls
     * (every destination is written by one source) */
#pragma omp parallel for num_threads(orc_threads)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int yy = y + C2Y[i];
                if (P->walls) {
                    if (yy < 0 || yy >= ny) continue; /* leaves through the wall */
                } else {
                    yy = wrap(yy, ny);
                }
                int xx = wrap(x + C2X[i], nx);
                f[i * N + yy * nx + xx] = w->fs[i * N + y * nx + x];
            }

    /* Zou-He no-slip wet-node walls: reconstruct the populations that would
     * have come from outside so that the wall velocity is zero */
    if (P->walls) {
        for (int x = 0; x < nx; ++x) {
            int n = x; /* bottom, unknowns 2, 5, 6 */
            double d = f[1 * N + n] - f[3 * N + n];
            f[2 * N + n] = f[4 * N + n];
            f[5 * N + n] = f[7 * N + n] - d / 2.0;
            f[6 * N + n] = f[8 * N + n] + d / 2.0;
            n = (ny - 1) * nx + x; /* top, unknowns 4, 7, 8 */
            d = f[1 * N + n] - f[3 * N + n];
            f[4 * N + n] = f[2 * N + n];
            f[7 * N + n] = f[5 * N + n] + d / 2.0;
            f[8 * N + n] = f[6 * N + n] - d / 2.0;
        }
    }
    memcpy(T, w->Tn, sizeof(double) * N);
}

static int d2q9_alloc(const orc_params *P, d2_work *w)
{
    size_t N = (size_t)P->nx * P->ny;
    double **fields[] = {&w->rho, &w->psi, &w->ux, &w->uy, &w->Fx, &w->Fy,
                         &w->Fix, &w->Fiy, &w->Tt, &w->Tn, &w->k1};
    for (size_t k = 0; k < sizeof fields / sizeof fields[0]; ++k) {
        *fields[k] = (double *)calloc(N, sizeof(double));
        if (!*fields[k]) return ORC_EINVAL;
    }
    w->fs = (double *)calloc(9 * N, sizeof(double));
    return w->fs ? ORC_OK : ORC_EINVAL;
}
static void d2q9_free(d2_work *w)
{
    free(w->rho); free(w->psi); free(w->ux); free(w->uy); free(w->Fx); free(w->Fy);
    free(w->Fix); free(w->Fiy); free(w->Tt); free(w->Tn); free(w->k1); free(w->fs);
}

/* ======================================================================
 * D1Q3 column (one wall-normal line; the x-uniform reduction of D2Q9 at
 * tau = 1).  Populations: 0 -> c = 0, 1 -> c = +1, 2 -> c = -1.
 * Weights 2/3, 1/6, 1/6; Shan-Chen weight w(1) = 1/2.
 * Equilibrium  f0 = 2/3 rho (1 - 3/2 u^2),  f+- = 1/6 rho (1 +- 3u + 3u^2).
 * Forcing at tau = 1 (the c_y-group sums of Li's scheme with Fx = ux = 0):
 *   F'_+- = (u F + sigma X'/6)/2 +- F/4,   F'_0 = -(u F + sigma X'/6).
 * ====================================================================== */
typedef struct {
    double *rho, *psi, *u, *F, *Fi, *Tt, *Tn, *k1, *fs;
} d1_work;

static double d1q3_energy_rhs(const orc_params *P, const double *Tf, const d1_work *w, int y)
{
    int ny = P->ny;
    int yp = wrap(y + 1, ny), ym = wrap(y - 1, ny);
    double gy = (Tf[yp] - Tf[ym]) / 2.0;
    double lap = Tf[yp] - 2.0 * Tf[y] + Tf[ym];
    double div = (w->u[yp] - w->u[ym]) / 2.0;
    double rho = w->rho[y];
    return -w->u[y] * gy + P->kappa / (rho * P->cv) * lap
           - Tf[y] / (rho * P->cv) * orc_eos_dpdT(P, rho, Tf[y]) * div;
}

static void d1q3_step_once(const orc_params *P, double *f, double *T, d1_work *w, int *flags,
                           orc_diag *dg)
{
    int ny = P->ny;
    double *f0 = f, *fp = f + ny, *fm = f + 2 * ny;
    for (int y = 0; y < ny; ++y) {
        w->rho[y] = f0[y] + fp[y] + fm[y];
        if (!(w->rho[y] == w->rho[y])) *flags |= ORC_FLAG_NAN;
        if (w->rho[y] <= 0) *flags |= ORC_FLAG_RHO;
    }
    double tot = 0;
    for (int y = 0; y < ny; ++y) tot += w->rho[y];
    double mean = tot / ny;
    for (int y = 0; y < ny; ++y) w->psi[y] = psi_of(P, w->rho[y], T[y], flags);
    for (int y = 0; y < ny; ++y) {
        int wall = P->walls && (y == 0 || y == ny - 1);
        if (wall) { w->Fi[y] = 0; w->F[y] = 0; continue; }
        double s = 0.5 * (w->psi[wrap(y + 1, ny)] - w->psi[wrap(y - 1, ny)]);
        w->Fi[y] = -P->G * w->psi[y] * s;
        double fg = gravity(P, w->rho[y], mean);
        w->F[y] = w->Fi[y] + fg;
    }
    double mass = 0, umax = 0, rmin = INFINITY;
    for (int y = 0; y < ny; ++y) {
        w->u[y] = (fp[y] - fm[y] + w->F[y] / 2.0) / w->rho[y];
        mass += w->rho[y];
        if (fabs(w->u[y]) > umax) umax = fabs(w->u[y]);
        if (w->rho[y] < rmin) rmin = w->rho[y];
    }
    dg->mass = mass; dg->mean_rho = mean; dg->max_u = umax; dg->min_rho = rmin;

    for (int y = 0; y < ny; ++y) {
        int wall = P->walls && (y == 0 || y == ny - 1);
        if (wall) { w->k1[y] = 0; w->Tt[y] = T[y]; continue; }
        w->k1[y] = d1q3_energy_rhs(P, T, w, y);
        w->Tt[y] = T[y] + w->k1[y];
    }
    for (int y = 0; y < ny; ++y) {
        int wall = P->walls && (y == 0 || y == ny - 1);
        if (wall) { w->Tn[y] = T[y]; continue; }
        double k2 = d1q3_energy_rhs(P, w->Tt, w, y);
        w->Tn[y] = T[y] + 0.5 * (w->k1[y] + k2);
    }
    /* collision at tau = 1: post-collision = equilibrium + forcing */
    for (int y = 0; y < ny; ++y) {
        double r = w->rho[y], u = w->u[y], F = w->F[y];
        double Xp = (w->Fi[y] != 0) ? w->Fi[y] * w->Fi[y] / (w->psi[y] * w->psi[y]) : 0.0;
        double q = u * F + P->sigma * Xp / 6.0;
        w->fs[y] = 2.0 * r / 3.0 * (1.0 - 1.5 * u * u) - q;
        w->fs[ny + y] = r / 6.0 * (1.0 + 3.0 * u + 3.0 * u * u) + q / 2.0 + F / 4.0;
        w->fs[2 * ny + y] = r / 6.0 * (1.0 - 3.0 * u + 3.0 * u * u) + q / 2.0 - F / 4.0;
    }
    /* stream */
    for (int y = 0; y < ny; ++y) {
        f0[y] = w->fs[y];
        int up = y + 1, dn = y - 1;
        if (P->walls) {
            if (up < ny) fp[up] = w->fs[ny + y];
            if (dn >= 0) fm[dn] = w->fs[2 * ny + y];
        } else {
            fp[wrap(up, ny)] = w->fs[ny + y];
            fm[wrap(dn, ny)] = w->fs[2 * ny + y];
        }
    }
    /* Zou-He (u = 0): the unknown population mirrors the known one */
    if (P->walls) {
        fp[0] = fm[0];
        fm[ny - 1] = fp[ny - 1];
    }
    memcpy(T, w->Tn, sizeof(double) * ny);
}

static int d1q3_alloc(const orc_params *P, d1_work *w)
{
    size_t N = (size_t)P->ny;
    double **fields[] = {&w->rho, &w->psi, &w->u, &w->F, &w->Fi, &w->Tt, &w->Tn, &w->k1};
    for (size_t k = 0; k < sizeof fields / sizeof fields[0]; ++k) {
        *fields[k] = (double *)calloc(N, sizeof(double));
        if (!*fields[k]) return ORC_EINVAL;
    }
    w->fs = (double *)calloc(3 * N, sizeof(double));
    return w->fs ? ORC_OK : ORC_EINVAL;
}
static void d1q3_free(d1_work *w)
{
    free(w->rho); free(w->psi); free(w->u); free(w->F); free(w->Fi);
    free(w->Tt); free(w->Tn); free(w->k1); free(w->fs);
}

static int tau_all_one(const orc_params *P)
{
    for (int k = 0; k < 6; ++k)
        if (P->tau[k] != 1.0) return 0;
    return 1;
}

/* forward declarations of the D3Q19 part (below) */
typedef struct d3_work d3_work;
static int d3q19_run(const orc_params *P, double *f, double *T, int64_t nsteps, int *flags,
                     orc_diag *dg);
static int d3q19_macro_out(const orc_params *P, const double *f, const double *T, double *rho,
                           double *ux, double *uy, double *uz, double *peos, double *pnn);
static int d3q19_collide_out(const orc_params *P, const double *f, const double *T, double *fstar);

/* ======================================================================
 * Public entry points
 * ====================================================================== */

/* rest populations f_i = w_i rho0 (the initial state of every run) */
int orc_init_rest(const orc_params *P, const double *rho0, double *f);

static int validate(const orc_params *P)
{
    if (P->lattice == 2 && (P->nx < 1 || P->ny < 3)) return ORC_EINVAL;
    if (P->lattice == 1 && P->ny < 3) return ORC_EINVAL;
    if (P->lattice == 3 && (P->nx < 1 || P->ny < 1 || P->nz < 3)) return ORC_EINVAL;
    if (P->lattice < 1 || P->lattice > 3) return ORC_EINVAL;
    for (int k = 0; k < 6; ++k)
        if (!(P->tau[k] > 0.5)) return ORC_EINVAL;
    if (P->lattice != 2 && !tau_all_one(P)) return ORC_EUNSUPPORTED;
    if (P->gravity_form < 1 || P->gravity_form > 3) return ORC_EINVAL;
    if (P->G == 0) return ORC_EINVAL;
    return ORC_OK;
}

/* Advance nsteps.  diag (may be NULL) receives the last step's level-n
 * diagnostics; its flags field is the OR over all steps. */
int orc_step(const orc_params *P, double *f, double *T, int64_t nsteps, orc_diag *diag)
{
    int rc = validate(P);
    if (rc) return rc;
    int flags = 0;
    orc_diag dg;
    memset(&dg, 0, sizeof dg);
    if (P->lattice == 2) {
        d2_work w;
        memset(&w, 0, sizeof w);
        if (d2q9_alloc(P, &w)) { d2q9_free(&w); return ORC_EINVAL; }
        for (int64_t s = 0; s < nsteps; ++s) d2q9_step_once(P, f, T, &w, &flags, &dg);
        d2q9_free(&w);
    } else if (P->lattice == 1) {
        d1_work w;
        memset(&w, 0, sizeof w);
        if (d1q3_alloc(P, &w)) { d1q3_free(&w); return ORC_EINVAL; }
        for (int64_t s = 0; s < nsteps; ++s) d1q3_step_once(P, f, T, &w, &flags, &dg);
        d1q3_free(&w);
    } else {
        rc = d3q19_run(P, f, T, nsteps, &flags, &dg);
        if (rc) return rc;
    }
    dg.flags = (double)flags;
    if (diag) *diag = dg;
    return ORC_OK;
}

/* Run a D1Q3 column (or any lattice) until max|u^n| < tol at a level n that
 * is a multiple of check_every, or until max_steps.  out3 = {steps taken,
 * status (0 converged, 1 diverged, 2 max_steps), unused}. */
int orc_run_to_steady(const orc_params *P, double *f, double *T, double tol, int64_t check_every,
                      int64_t max_steps, double *out3)
{
    int rc = validate(P);
    if (rc) return rc;
    if (check_every < 1) return ORC_EINVAL;
    int64_t n = 0;
    int status = 2;
    for (;;) {
        /* a step reports the diagnostics of the level it starts from */
        if (n >= max_steps) { status = 2; break; }
        orc_diag dg;
        /* keep a copy of level n so that a converged run returns it */
        size_t N = P->lattice == 1   ? (size_t)P->ny
                   : P->lattice == 2 ? (size_t)P->nx * P->ny
                                     : (size_t)P->nx * P->ny * P->nz;
        int Q = P->lattice == 1 ? 3 : P->lattice == 2 ? 9 : 19;
        double *fc = NULL, *Tc = NULL;
        int check = (n % check_every) == 0;
        if (check) {
            fc = (double *)malloc(sizeof(double) * Q * N);
            Tc = (double *)malloc(sizeof(double) * N);
            memcpy(fc, f, sizeof(double) * Q * N);
            memcpy(Tc, T, sizeof(double) * N);
        }
        rc = orc_step(P, f, T, 1, &dg);
        if (rc) { free(fc); free(Tc); return rc; }
        if (((int)dg.flags) != 0 || !(dg.max_u == dg.max_u)) {
            status = 1;
            free(fc); free(Tc);
            break;
        }
        if (check && dg.max_u < tol) {
            memcpy(f, fc, sizeof(double) * Q * N);
            memcpy(T, Tc, sizeof(double) * N);
            free(fc); free(Tc);
            status = 0;
            break;
        }
        free(fc); free(Tc);
        ++n;
    }
    out3[0] = (double)n;
    out3[1] = (double)status;
    out3[2] = 0;
    return ORC_OK;
}

/* Macroscopic readout of time level n: rho, u, T-independent p_EOS and the
 * normal pressure p_nn (the wall-normal diagonal entry of Eq.
 * GeneralPressureTensor) with plain central differences, interior nodes
 * only; wall nodes report p_EOS.  Any output pointer may be NULL. */
int orc_macro(const orc_params *P, const double *f, const double *T, double *rho, double *ux,
              double *uy, double *uz, double *peos, double *pnn)
{
    int rc = validate(P);
    if (rc) return rc;
    int flags = 0;
    if (P->lattice == 3) return d3q19_macro_out(P, f, T, rho, ux, uy, uz, peos, pnn);
    if (P->lattice == 2) {
        int nx = P->nx, ny = P->ny;
        d2_work w;
        memset(&w, 0, sizeof w);
        if (d2q9_alloc(P, &w)) { d2q9_free(&w); return ORC_EINVAL; }
        d2q9_macro(P, f, T, &w, &flags);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int n = y * nx + x;
                if (rho) rho[n] = w.rho[n];
                if (ux) ux[n] = w.ux[n];
                if (uy) uy[n] = w.uy[n];
                if (uz) uz[n] = 0;
                double pe = orc_eos_p(P, w.rho[n], T[n]);
                if (peos) peos[n] = pe;
                if (pnn) {
                    int wall = P->walls && (y == 0 || y == ny - 1);
                    if (wall) { pnn[n] = pe; continue; }
                    double ps = w.psi[n];
                    double pxp = w.psi[y * nx + wrap(x + 1, nx)], pxm = w.psi[y * nx + wrap(x - 1, nx)];
                    double pyp = w.psi[wrap(y + 1, ny) * nx + x], pym = w.psi[wrap(y - 1, ny) * nx + x];
                    double dx = (pxp - pxm) / 2.0, dy = (pyp - pym) / 2.0;
                    double lap = pxp + pxm + pyp + pym - 4.0 * ps;
                    double dyy = pyp - 2.0 * ps + pym;
                    pnn[n] = pe + P->sigma * P->G * P->G / 6.0 * (dx * dx + dy * dy)
                             + P->G / 12.0 * ps * lap + P->G / 6.0 * ps * dyy;
                }
            }
        d2q9_free(&w);
        return ORC_OK;
    }
    /* D1Q3 */
    int ny = P->ny;
    d1_work w;
    memset(&w, 0, sizeof w);
    if (d1q3_alloc(P, &w)) { d1q3_free(&w); return ORC_EINVAL; }
    orc_diag dg;
    /* the level-n fields are the ones one step computes before collision;
     * evaluate them on a copy so that f and T stay untouched */
    double *fc = (double *)malloc(sizeof(double) * 3 * ny);
    double *Tc = (double *)malloc(sizeof(double) * ny);
    memcpy(fc, f, sizeof(double) * 3 * ny);
    memcpy(Tc, T, sizeof(double) * ny);
    d1q3_step_once(P, fc, Tc, &w, &flags, &dg);
    for (int y = 0; y < ny; ++y) {
        if (rho) rho[y] = w.rho[y];
        if (ux) ux[y] = 0;
        if (uy) uy[y] = w.u[y];
        if (uz) uz[y] = 0;
        double pe = orc_eos_p(P, w.rho[y], T[y]);
        if (peos) peos[y] = pe;
        if (pnn) {
            int wall = P->walls && (y == 0 || y == ny - 1);
            if (wall) { pnn[y] = pe; continue; }
            double ps = w.psi[y], pp = w.psi[wrap(y + 1, ny)], pm = w.psi[wrap(y - 1, ny)];
            double dy = (pp - pm) / 2.0, dyy = pp - 2.0 * ps + pm;
            pnn[y] = pe + P->sigma * P->G * P->G / 6.0 * dy * dy + P->G / 12.0 * ps * dyy
                     + P->G / 6.0 * ps * dyy;
        }
    }
    free(fc); free(Tc);
    d1q3_free(&w);
    return ORC_OK;
}

/* One collision without streaming, for the algebra tests: fstar receives the
 * post-collision populations of every node (D2Q9, D1Q3 and D3Q19). */
int orc_collide(const orc_params *P, const double *f, const double *T, double *fstar)
{
    int rc = validate(P);
    if (rc) return rc;
    int flags = 0;
    orc_diag dg;
    if (P->lattice == 2) {
        int N = P->nx * P->ny;
        d2_work w;
        memset(&w, 0, sizeof w);
        if (d2q9_alloc(P, &w)) { d2q9_free(&w); return ORC_EINVAL; }
        double *fc = (double *)malloc(sizeof(double) * 9 * N);
        double *Tc = (double *)malloc(sizeof(double) * N);
        memcpy(fc, f, sizeof(double) * 9 * N);
        memcpy(Tc, T, sizeof(double) * N);
        d2q9_step_once(P, fc, Tc, &w, &flags, &dg);
        memcpy(fstar, w.fs, sizeof(double) * 9 * N);
        free(fc); free(Tc);
        d2q9_free(&w);
        return ORC_OK;
    }
    if (P->lattice == 1) {
        int ny = P->ny;
        d1_work w;
        memset(&w, 0, sizeof w);
        if (d1q3_alloc(P, &w)) { d1q3_free(&w); return ORC_EINVAL; }
        double *fc = (double *)malloc(sizeof(double) * 3 * ny);
        double *Tc = (double *)malloc(sizeof(double) * ny);
        memcpy(fc, f, sizeof(double) * 3 * ny);
        memcpy(Tc, T, sizeof(double) * ny);
        d1q3_step_once(P, fc, Tc, &w, &flags, &dg);
        memcpy(fstar, w.fs, sizeof(double) * 3 * ny);
        free(fc); free(Tc);
        d1q3_free(&w);
        return ORC_OK;
    }
    if (P->lattice == 3) return d3q19_collide_out(P, f, T, fstar);
    return ORC_EUNSUPPORTED;
}

/* ======================================================================
 * D3Q19 (an extension beyond the paper's D2Q9; tau = 1 only, where every
 * MRT relaxation rate is one and the collision is the BGK one).
 * Velocities: rest, 6 axis neighbours, 12 edge neighbours.  Weights 1/3,
 * 1/18, 1/36.  Shan-Chen weights w(1) = 1/6, w(2) = 1/12 so that
 * sum_i w c_a c_b = delta_ab as for the D2Q9 weights.  Forcing at tau = 1:
 * half of Guo's term plus the isotropic sigma term
 * w_i (|c_i|^2 - 1) (3/4) sigma X', which is the D2Q9 sigma term of Li's
 * scheme written without reference to the 2-D moment basis.
 * ====================================================================== */
static int C3X[19], C3Y[19], C3Z[19];
static double W3[19];
static double W3DEN[19]; /* w_i = 1 / W3DEN[i] */
static int d3_ready = 0;
static void d3_init(void)
{
    if (d3_ready) return;
    int k = 0;
    C3X[k] = C3Y[k] = C3Z[k] = 0; W3[k] = 1.0 / 3.0; ++k;
    for (int x = -1; x <= 1; ++x)
        for (int y = -1; y <= 1; ++y)
            for (int z = -1; z <= 1; ++z) {
                int c2 = x * x + y * y + z * z;
                if (c2 == 1) { C3X[k] = x; C3Y[k] = y; C3Z[k] = z; W3[k] = 1.0 / 18.0; ++k; }
            }
    for (int x = -1; x <= 1; ++x)
        for (int y = -1; y <= 1; ++y)
            for (int z = -1; z <= 1; ++z) {
                int c2 = x * x + y * y + z * z;
                if (c2 == 2) { C3X[k] = x; C3Y[k] = y; C3Z[k] = z; W3[k] = 1.0 / 36.0; ++k; }
            }
    for (int i = 0; i < 19; ++i) W3DEN[i] = (i == 0) ? 3.0 : (i < 7 ? 18.0 : 36.0);
    d3_ready = 1;
}
void orc_d3q19_velocities(int *out57, double *w19)
{
    d3_init();
    for (int i = 0; i < 19; ++i) {
        out57[3 * i] = C3X[i]; out57[3 * i + 1] = C3Y[i]; out57[3 * i + 2] = C3Z[i];
        w19[i] = W3[i];
    }
}
static int opp3(int i)
{
    for (int j = 0; j < 19; ++j)
        if (C3X[j] == -C3X[i] && C3Y[j] == -C3Y[i] && C3Z[j] == -C3Z[i]) return j;
    return -1;
}
static int find3(int x, int y, int z)
{
    for (int j = 0; j < 19; ++j)
        if (C3X[j] == x && C3Y[j] == y && C3Z[j] == z) return j;
    return -1;
}

struct d3_work {
    double *rho, *psi, *ux, *uy, *uz, *Fx, *Fy, *Fz, *Fi2, *Tt, *Tn, *k1, *fs;
};

static size_t idx3(const orc_params *P, int x, int y, int z)
{
    return ((size_t)z * P->ny + y) * P->nx + x;
}

static double d3q19_macro(const orc_params *P, const double *f, const double *T, d3_work *w,
                          int *flags)
{
    int nx = P->nx, ny = P->ny, nz = P->nz;
    size_t N = (size_t)nx * ny * nz;
    int fl = 0;
#pragma omp parallel for num_threads(orc_threads) reduction(| : fl)
    for (size_t n = 0; n < N; ++n) {
        double s = 0;
        for (int i = 0; i < 19; ++i) s += f[i * N + n];
        w->rho[n] = s;
        if (!(s == s)) fl |= ORC_FLAG_NAN;
        if (s <= 0) fl |= ORC_FLAG_RHO;
    }
    double tot = 0;
    for (size_t n = 0; n < N; ++n) tot += w->rho[n];
    double mean = tot / (double)N;
#pragma omp parallel for num_threads(orc_threads) reduction(| : fl)
    for (size_t n = 0; n < N; ++n) w->psi[n] = psi_of(P, w->rho[n], T[n], &fl);
    *flags |= fl;
#pragma omp parallel for num_threads(orc_threads)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = idx3(P, x, y, z);
                int wall = P->walls && (z == 0 || z == nz - 1);
                if (wall) {
                    w->Fx[n] = w->Fy[n] = w->Fz[n] = w->Fi2[n] = 0;
                    continue;
                }
                double sx = 0, sy = 0, sz = 0;
                for (int i = 1; i < 19; ++i) {
                    int c2 = C3X[i] * C3X[i] + C3Y[i] * C3Y[i] + C3Z[i] * C3Z[i];
                    double wsc = (c2 == 1) ? 1.0 / 6.0 : 1.0 / 12.0;
                    double ps = w->psi[idx3(P, wrap(x + C3X[i], nx), wrap(y + C3Y[i], ny),
                                            wrap(z + C3Z[i], nz))];
                    sx += wsc * ps * C3X[i];
                    sy += wsc * ps * C3Y[i];
                    sz += wsc * ps * C3Z[i];
                }
                double fix = -P->G * w->psi[n] * sx;
                double fiy = -P->G * w->psi[n] * sy;
                double fiz = -P->G * w->psi[n] * sz;
                double fg = gravity(P, w->rho[n], mean);
                w->Fx[n] = fix;
                w->Fy[n] = fiy;
                w->Fz[n] = fiz + fg;
                w->Fi2[n] = fix * fix + fiy * fiy + fiz * fiz;
            }
#pragma omp parallel for num_threads(orc_threads)
    for (size_t n = 0; n < N; ++n) {
        double jx = 0, jy = 0, jz = 0;
        for (int i = 0; i < 19; ++i) {
            jx += f[i * N + n] * C3X[i];
            jy += f[i * N + n] * C3Y[i];
            jz += f[i * N + n] * C3Z[i];
        }
        w->ux[n] = (jx + w->Fx[n] / 2.0) / w->rho[n];
        w->uy[n] = (jy + w->Fy[n] / 2.0) / w->rho[n];
        w->uz[n] = (jz + w->Fz[n] / 2.0) / w->rho[n];
    }
    return mean;
}

static double d3q19_energy_rhs(const orc_params *P, const double *Tf, const d3_work *w, int x,
                               int y, int z)
{
    size_t n = idx3(P, x, y, z);
    double gx = 0, gy = 0, gz = 0, lap = 0, div = 0;
    for (int i = 0; i < 19; ++i) {
        size_t m = idx3(P, wrap(x + C3X[i], P->nx), wrap(y + C3Y[i], P->ny),
                        wrap(z + C3Z[i], P->nz));
        gx += W3[i] * C3X[i] * Tf[m];
        gy += W3[i] * C3Y[i] * Tf[m];
        gz += W3[i] * C3Z[i] * Tf[m];
        lap += W3[i] * (Tf[m] - Tf[n]);
        div += W3[i] * (C3X[i] * w->ux[m] + C3Y[i] * w->uy[m] + C3Z[i] * w->uz[m]);
    }
    gx *= 3.0; gy *= 3.0; gz *= 3.0; lap *= 6.0; div *= 3.0;
    double rho = w->rho[n];
    return -(w->ux[n] * gx + w->uy[n] * gy + w->uz[n] * gz) + P->kappa / (rho * P->cv) * lap
           - Tf[n] / (rho * P->cv) * orc_eos_dpdT(P, rho, Tf[n]) * div;
}

static void d3q19_step_once(const orc_params *P, double *f, double *T, d3_work *w, int *flags,
                            orc_diag *dg)
{
    int nx = P->nx, ny = P->ny, nz = P->nz;
    size_t N = (size_t)nx * ny * nz;
    double mean = d3q19_macro(P, f, T, w, flags);
    double mass = 0, umax = 0, rmin = INFINITY;
    for (size_t n = 0; n < N; ++n) {
        mass += w->rho[n];
        double um = sqrt(w->ux[n] * w->ux[n] + w->uy[n] * w->uy[n] + w->uz[n] * w->uz[n]);
        if (um > umax) umax = um;
        if (w->rho[n] < rmin) rmin = w->rho[n];
    }
    dg->mass = mass; dg->mean_rho = mean; dg->max_u = umax; dg->min_rho = rmin;
#pragma omp parallel for num_threads(orc_threads)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = idx3(P, x, y, z);
                int wall = P->walls && (z == 0 || z == nz - 1);
                if (wall) { w->k1[n] = 0; w->Tt[n] = T[n]; continue; }
                w->k1[n] = d3q19_energy_rhs(P, T, w, x, y, z);
                w->Tt[n] = T[n] + w->k1[n];
            }
#pragma omp parallel for num_threads(orc_threads)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = idx3(P, x, y, z);
                int wall = P->walls && (z == 0 || z == nz - 1);
                if (wall) { w->Tn[n] = T[n]; continue; }
                double k2 = d3q19_energy_rhs(P, w->Tt, w, x, y, z);
                w->Tn[n] = T[n] + 0.5 * (w->k1[n] + k2);
            }
    /* collision at tau = 1: f* = f_eq + F' */
#pragma omp parallel for num_threads(orc_threads)
    for (size_t n = 0; n < N; ++n) {
        double r = w->rho[n], ux = w->ux[n], uy = w->uy[n], uz = w->uz[n];
        double Fx = w->Fx[n], Fy = w->Fy[n], Fz = w->Fz[n];
        double Xp = (w->Fi2[n] > 0) ? w->Fi2[n] / (w->psi[n] * w->psi[n]) : 0.0;
        double uu = ux * ux + uy * uy + uz * uz;
        for (int i = 0; i < 19; ++i) {
            double cu = C3X[i] * ux + C3Y[i] * uy + C3Z[i] * uz;
            double cF = C3X[i] * Fx + C3Y[i] * Fy + C3Z[i] * Fz;
            double uF = ux * Fx + uy * Fy + uz * Fz;
            double feq = r / W3DEN[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            /* Guo: (1 - 1/(2 tau)) w_i [3 (c - u).F + 9 (c.u)(c.F)] at tau = 1 */
            double guo = 0.5 * W3[i] * (3.0 * (cF - uF) + 9.0 * cu * cF);
            int c2 = C3X[i] * C3X[i] + C3Y[i] * C3Y[i] + C3Z[i] * C3Z[i];
            double sig = W3[i] * (c2 - 1.0) * 0.75 * P->sigma * Xp;
            w->fs[i * N + n] = feq + guo + sig;
        }
    }
    /* stream: periodic in x and y; z periodic or cut at the walls (every
     * destination is written by one source) */
#pragma omp parallel for num_threads(orc_threads)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                for (int i = 0; i < 19; ++i) {
                    int zz = z + C3Z[i];
                    if (P->walls) {
                        if (zz < 0 || zz >= nz) continue;
                    } else {
                        zz = wrap(zz, nz);
                    }
                    size_t to = idx3(P, wrap(x + C3X[i], nx), wrap(y + C3Y[i], ny), zz);
                    f[i * N + to] = w->fs[i * N + idx3(P, x, y, z)];
                }
    /* Zou-He wet-node walls with zero velocity (the D3Q19 form with
     * transverse momentum corrections) */
    if (P->walls) {
        for (int side = 0; side < 2; ++side) {
            int z = side == 0 ? 0 : nz - 1;
            int s = side == 0 ? 1 : -1; /* direction of the unknown populations */
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t n = idx3(P, x, y, z);
                    /* transverse momentum of the in-plane populations */
                    double Nx = 0, Ny = 0;
                    for (int i = 0; i < 19; ++i)
                        if (C3Z[i] == 0) {
                            Nx += 0.5 * C3X[i] * f[i * N + n];
                            Ny += 0.5 * C3Y[i] * f[i * N + n];
                        }
                    int iz = find3(0, 0, s);
                    f[iz * N + n] = f[opp3(iz) * N + n];
                    int ixp = find3(1, 0, s), ixm = find3(-1, 0, s);
                    int iyp = find3(0, 1, s), iym = find3(0, -1, s);
                    f[ixp * N + n] = f[opp3(ixp) * N + n] - Nx;
                    f[ixm * N + n] = f[opp3(ixm) * N + n] + Nx;
                    f[iyp * N + n] = f[opp3(iyp) * N + n] - Ny;
                    f[iym * N + n] = f[opp3(iym) * N + n] + Ny;
                }
        }
    }
    memcpy(T, w->Tn, sizeof(double) * N);
}

static int d3q19_alloc(const orc_params *P, d3_work *w)
{
    size_t N = (size_t)P->nx * P->ny * P->nz;
    double **fields[] = {&w->rho, &w->psi, &w->ux, &w->uy, &w->uz, &w->Fx, &w->Fy,
                         &w->Fz, &w->Fi2, &w->Tt, &w->Tn, &w->k1};
    for (size_t k = 0; k < sizeof fields / sizeof fields[0]; ++k) {
        *fields[k] = (double *)calloc(N, sizeof(double));
        if (!*fields[k]) return ORC_EINVAL;
    }
    w->fs = (double *)calloc(19 * N, sizeof(double));
    return w->fs ? ORC_OK : ORC_EINVAL;
}
static void d3q19_free(d3_work *w)
{
    free(w->rho); free(w->psi); free(w->ux); free(w->uy); free(w->uz); free(w->Fx);
    free(w->Fy); free(w->Fz); free(w->Fi2); free(w->Tt); free(w->Tn); free(w->k1); free(w->fs);
}

static int d3q19_run(const orc_params *P, double *f, double *T, int64_t nsteps, int *flags,
                     orc_diag *dg)
{
    d3_init();
    d3_work w;
    memset(&w, 0, sizeof w);
    if (d3q19_alloc(P, &w)) { d3q19_free(&w); return ORC_EINVAL; }
    for (int64_t s = 0; s < nsteps; ++s) d3q19_step_once(P, f, T, &w, flags, dg);
    d3q19_free(&w);
    return ORC_OK;
}

/* the post-collision populations of one step (the step's own intermediate,
 * taken on copies of f and T) */
static int d3q19_collide_out(const orc_params *P, const double *f, const double *T, double *fstar)
{
    d3_init();
    size_t N = (size_t)P->nx * P->ny * P->nz;
    int flags = 0;
    orc_diag dg;
    d3_work w;
    memset(&w, 0, sizeof w);
    if (d3q19_alloc(P, &w)) { d3q19_free(&w); return ORC_EINVAL; }
    double *fc = (double *)malloc(sizeof(double) * 19 * N);
    double *Tc = (double *)malloc(sizeof(double) * N);
    memcpy(fc, f, sizeof(double) * 19 * N);
    memcpy(Tc, T, sizeof(double) * N);
    d3q19_step_once(P, fc, Tc, &w, &flags, &dg);
    memcpy(fstar, w.fs, sizeof(double) * 19 * N);
    free(fc); free(Tc);
    d3q19_free(&w);
    return ORC_OK;
}

static int d3q19_macro_out(const orc_params *P, const double *f, const double *T, double *rho,
                           double *ux, double *uy, double *uz, double *peos, double *pnn)
{
    d3_init();
    int nx = P->nx, ny = P->ny, nz = P->nz;
    int flags = 0;
    d3_work w;
    memset(&w, 0, sizeof w);
    if (d3q19_alloc(P, &w)) { d3q19_free(&w); return ORC_EINVAL; }
    d3q19_macro(P, f, T, &w, &flags);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t n = idx3(P, x, y, z);
                if (rho) rho[n] = w.rho[n];
                if (ux) ux[n] = w.ux[n];
                if (uy) uy[n] = w.uy[n];
                if (uz) uz[n] = w.uz[n];
                double pe = orc_eos_p(P, w.rho[n], T[n]);
                if (peos) peos[n] = pe;
                if (pnn) {
                    int wall = P->walls && (z == 0 || z == nz - 1);
                    if (wall) { pnn[n] = pe; continue; }
                    double ps = w.psi[n];
                    double pxp = w.psi[idx3(P, wrap(x + 1, nx), y, z)];
                    double pxm = w.psi[idx3(P, wrap(x - 1, nx), y, z)];
                    double pyp = w.psi[idx3(P, x, wrap(y + 1, ny), z)];
                    double pym = w.psi[idx3(P, x, wrap(y - 1, ny), z)];
                    double pzp = w.psi[idx3(P, x, y, wrap(z + 1, nz))];
                    double pzm = w.psi[idx3(P, x, y, wrap(z - 1, nz))];
                    double dx = (pxp - pxm) / 2.0, dy = (pyp - pym) / 2.0, dz = (pzp - pzm) / 2.0;
                    double lap = pxp + pxm + pyp + pym + pzp + pzm - 6.0 * ps;
                    double dzz = pzp - 2.0 * ps + pzm;
                    pnn[n] = pe + P->sigma * P->G * P->G / 6.0 * (dx * dx + dy * dy + dz * dz)
                             + P->G / 12.0 * ps * lap + P->G / 6.0 * ps * dzz;
                }
            }
    d3q19_free(&w);
    return ORC_OK;
}

int orc_init_rest(const orc_params *P, const double *rho0, double *f)
{
    int rc = validate(P);
    if (rc) return rc;
    if (P->lattice == 2) {
        size_t N = (size_t)P->nx * P->ny;
        for (int i = 0; i < 9; ++i)
            for (size_t n = 0; n < N; ++n) f[i * N + n] = W2[i] * rho0[n];
    } else if (P->lattice == 1) {
        size_t N = (size_t)P->ny;
        const double w1[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
        for (int i = 0; i < 3; ++i)
            for (size_t n = 0; n < N; ++n) f[i * N + n] = w1[i] * rho0[n];
    } else {
        d3_init();
        size_t N = (size_t)P->nx * P->ny * P->nz;
        for (int i = 0; i < 19; ++i)
            for (size_t n = 0; n < N; ++n) f[i * N + n] = W3[i] * rho0[n];
    }
    return ORC_OK;
}
