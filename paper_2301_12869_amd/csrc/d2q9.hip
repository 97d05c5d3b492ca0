// D2Q9 fused lattice update for gfx950: one launch per time step.
//
// State between launches: post-collision populations f* of the previous step
// (structure of arrays, plane i holds population i over y*nx + x), and T^n.
// One launch does, for a TX x TY tile of nodes (Sec. III of the paper):
//   phase 1, tile + 3-node halo: pull-stream f^n_i(x) = f*_i(x - c_i) with
//            Zou-He reconstruction of the unknown populations at wall nodes,
//            rho = sum f_i (Eq. Density), j = sum f_i c_i, psi(rho, T^n)
//            (Eqs. EOS, InteractionPotential)                   -> LDS
//   phase 2, tile + 2: Shan-Chen force (Eq. ShanChenForce, zero at walls),
//            gravity (Eq. Gravity_1 or Gravity_2, zero at walls), force-
//            corrected velocity u = (j + F/2)/rho (Eq. Momentum)  -> LDS
//   phase 3, tile + 1: first Heun stage of Eq. Energy_Equation with
//            isotropic differences: k1 = K(T^n)                  -> LDS
//   phase 4, tile:     T~ = T^n + k1, T^{n+1} = T^n + (k1 + K(T~))/2; MRT
//            collision with Li's forcing (Eqs. OperatorMRT, LiFS), or at
//            tau = 1 its closed form f* = f_eq + F'; store f* and T^{n+1};
//            block partials of the next level's mass (each f*_i weighted by
//            how many times it will be counted after streaming and the wall
//            reconstruction), of max |u|, min rho and the flags.
// The last block to finish reduces the partials in block order and writes
// <rho> of the next level, which is what the next launch's gravity form 2
// uses: no second pass over the populations is needed for the mean.
#include <hip/hip_runtime.h>

#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {

constexpr int kThreads = 256;

template <class S>
struct PopIO;
template <>
struct PopIO<double> {
    __device__ static __forceinline__ double load(const double *p, size_t i, double /*wref*/)
    {
        return p[i];
    }
    __device__ static __forceinline__ double store(double *p, size_t i, double v, double)
    {
        p[i] = v;
        return v;
    }
};
template <>
struct PopIO<float> {
    // FP32 deviation storage: the stored value is f_i - w_i rho_ref
    __device__ static __forceinline__ double load(const float *p, size_t i, double wref)
    {
        return wref + (double)p[i];
    }
    __device__ static __forceinline__ double store(float *p, size_t i, double v, double wref)
    {
        const float d = (float)(v - wref);
        p[i] = d;
        return wref + (double)d;  // the value the next step will read
    }
};

constexpr double kW0 = 4.0 / 9.0, kW1 = 1.0 / 9.0, kW5 = 1.0 / 36.0;

// Isotropic second-order differences on the D2Q9 stencil (weights w_i/c_s^2)
// of a field held in LDS with row stride `ld`, centred at index c.
struct Stencil {
    double e, w, n, s, ne, nw, sw, se;
    __device__ __forceinline__ void load(const double *a, int c, int ld)
    {
        e = a[c + 1]; w = a[c - 1]; n = a[c + ld]; s = a[c - ld];
        ne = a[c + ld + 1]; nw = a[c + ld - 1]; sw = a[c - ld - 1]; se = a[c - ld + 1];
    }
    // 3 sum_i w_i c_ix phi_i
    __device__ __forceinline__ double dx() const
    {
        return (e - w) * (1.0 / 3.0) + ((ne + se) - (nw + sw)) * (1.0 / 12.0);
    }
    __device__ __forceinline__ double dy() const
    {
        return (n - s) * (1.0 / 3.0) + ((ne + nw) - (se + sw)) * (1.0 / 12.0);
    }
    // 6 sum_i w_i (phi_i - phi_0), as differences so that it vanishes
    // exactly on a uniform field
    __device__ __forceinline__ double lap(double c0) const
    {
        return (((e - c0) + (w - c0)) + ((n - c0) + (s - c0))) * (2.0 / 3.0) +
               (((ne - c0) + (nw - c0)) + ((sw - c0) + (se - c0))) * (1.0 / 6.0);
    }
};

// Right-hand side of the energy equation at one node, for the field whose
// stencil values are in t and centre value is T0.
__device__ __forceinline__ double energy_rhs(const Phys &c, const Stencil &t, double T0, double ux,
                                             double uy, double divu, double inv_rho, double Z)
{
    const double adv = -(ux * t.dx() + uy * t.dy());
    const double cond = c.kappa_over_cv * inv_rho * t.lap(T0);
    const double work = -T0 * c.R_over_cv * Z * divu;
    return adv + cond + work;
}

__device__ __forceinline__ double divergence(const double *ux, const double *uy, int c, int ld)
{
    Stencil a, b;
    a.load(ux, c, ld);
    b.load(uy, c, ld);
    return a.dx() + b.dy();
}

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <class S, bool TAU1, bool WALLS, int TX, int TY>
__global__ __launch_bounds__(kThreads) void d2q9_step(const S *__restrict__ fin,
                                                      S *__restrict__ fout,
                                                      const double *__restrict__ Tin,
                                                      double *__restrict__ Tout, Phys c,
                                                      int nx, int ny, int tiles_x,
                                                      double *__restrict__ partials,
                                                      StepState *__restrict__ st,
                                                      int64_t step)
{
    constexpr int W3 = TX + 6, H3 = TY + 6;
    constexpr int W2 = TX + 4, H2 = TY + 4;
    constexpr int W1 = TX + 2, H1 = TY + 2;
    __shared__ double s_psi[H3 * W3];
    __shared__ double s_rho[H2 * W2];
    __shared__ double s_T[H2 * W2];
    __shared__ double s_ux[H2 * W2];
    __shared__ double s_uy[H2 * W2];
    __shared__ double s_k1[H1 * W1];  // first Heun stage K(T^n); T~ = T^n + k1
    __shared__ double s_red[4 * kThreads / 64];
    __shared__ unsigned s_ured[kThreads / 64];

    const int tid = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (tile % tiles_x) * TX;
    const int y0 = (tile / tiles_x) * TY;
    const size_t N = (size_t)nx * ny;
    const double rr = c.rho_ref;
    const double mean = st->mean[step & 1];

    // ---- phase 1: pull, density, momentum, pseudopotential on tile + 3 ----
    for (int r = tid; r < H3 * W3; r += kThreads) {
        const int ry = r / W3, rx = r - ry * W3;
        int gy = y0 + ry - 3;
        const int gx = wrapi(x0 + rx - 3, nx);
        bool valid = true;
        if (WALLS)
            valid = (gy >= 0 && gy < ny);
        else
            gy = wrapi(gy, ny);
        double rho = 0.0, jx = 0.0, jy = 0.0, psi = 0.0, T = 0.0;
        if (valid) {
            const int xm = (gx == 0) ? nx - 1 : gx - 1;
            const int xp = (gx == nx - 1) ? 0 : gx + 1;
            int ym = gy - 1, yp = gy + 1;
            if (!WALLS) {
                ym = (gy == 0) ? ny - 1 : ym;
                yp = (gy == ny - 1) ? 0 : yp;
            }
            const bool bot = WALLS && gy == 0, top = WALLS && gy == ny - 1;
            const size_t row = (size_t)gy * nx;
            const size_t rowm = (size_t)(bot ? gy : ym) * nx;  // never read when bot
            const size_t rowp = (size_t)(top ? gy : yp) * nx;  // never read when top
            double f0 = PopIO<S>::load(fin, 0 * N + row + gx, kW0 * rr);
            double f1 = PopIO<S>::load(fin, 1 * N + row + xm, kW1 * rr);
            double f3 = PopIO<S>::load(fin, 3 * N + row + xp, kW1 * rr);
            double f2 = 0.0, f4 = 0.0, f5 = 0.0, f6 = 0.0, f7 = 0.0, f8 = 0.0;
            if (!bot) {
                f2 = PopIO<S>::load(fin, 2 * N + rowm + gx, kW1 * rr);
                f5 = PopIO<S>::load(fin, 5 * N + rowm + xm, kW5 * rr);
                f6 = PopIO<S>::load(fin, 6 * N + rowm + xp, kW5 * rr);
            }
            if (!top) {
                f4 = PopIO<S>::load(fin, 4 * N + rowp + gx, kW1 * rr);
                f7 = PopIO<S>::load(fin, 7 * N + rowp + xp, kW5 * rr);
                f8 = PopIO<S>::load(fin, 8 * N + rowp + xm, kW5 * rr);
            }
            if (bot) {  // Zou-He, zero wall velocity: unknowns 2, 5, 6
                const double d = f1 - f3;
                f2 = f4;
                f5 = f7 - 0.5 * d;
                f6 = f8 + 0.5 * d;
            }
            if (top) {  // unknowns 4, 7, 8
                const double d = f1 - f3;
                f4 = f2;
                f7 = f5 + 0.5 * d;
                f8 = f6 - 0.5 * d;
            }
            rho = ((f0 + f1) + (f2 + f3)) + ((f4 + f5) + (f6 + f7)) + f8;
            jx = (f1 - f3) + (f5 - f6) + (f8 - f7);
            jy = (f2 - f4) + (f5 + f6) - (f7 + f8);
            T = Tin[row + gx];
            double Zdummy;
            psi = psi_and_Z(c, rho, T, Zdummy);
        }
        s_psi[r] = psi;
        if (rx >= 1 && rx < W3 - 1 && ry >= 1 && ry < H3 - 1) {
            const int q = (ry - 1) * W2 + (rx - 1);
            s_rho[q] = rho;
            s_T[q] = T;
            s_ux[q] = jx;
            s_uy[q] = jy;
        }
    }
    __syncthreads();

    // ---- phase 2: force and force-corrected velocity on tile + 2 ----
    for (int r = tid; r < H2 * W2; r += kThreads) {
        const int ry = r / W2, rx = r - ry * W2;
        int gy = y0 + ry - 2;
        bool valid = true, wall = false;
        if (WALLS) {
            valid = (gy >= 0 && gy < ny);
            wall = (gy == 0 || gy == ny - 1);
        }
        if (!valid) continue;
        const double rho = s_rho[r];
        double Fx = 0.0, Fy = 0.0;
        if (!wall) {
            Stencil p;
            const int c3 = (ry + 1) * W3 + (rx + 1);
            p.load(s_psi, c3, W3);
            // sum_i w(|c_i|^2) psi(x + c_i) c_i with w(1) = 1/3, w(2) = 1/12
            const double sx = (p.e - p.w) * (1.0 / 3.0) + ((p.ne + p.se) - (p.nw + p.sw)) * (1.0 / 12.0);
            const double sy = (p.n - p.s) * (1.0 / 3.0) + ((p.ne + p.nw) - (p.se + p.sw)) * (1.0 / 12.0);
            const double mg = -c.G * s_psi[c3];
            const double fg = (c.form == 2) ? -(rho - mean) * c.g : -rho * c.g;
            Fx = mg * sx;
            Fy = mg * sy + fg;
        }
        const double inv = 1.0 / rho;
        s_ux[r] = (s_ux[r] + 0.5 * Fx) * inv;
        s_uy[r] = (s_uy[r] + 0.5 * Fy) * inv;
    }
    __syncthreads();

    // ---- phase 3: first Heun stage on tile + 1 ----
    for (int r = tid; r < H1 * W1; r += kThreads) {
        const int ry = r / W1, rx = r - ry * W1;
        const int gy = y0 + ry - 1;
        const int c2 = (ry + 1) * W2 + (rx + 1);
        if (WALLS && (gy < 0 || gy >= ny || gy == 0 || gy == ny - 1)) {
            s_k1[r] = 0.0;  // Dirichlet walls: T~ = T
            continue;
        }
        const double rho = s_rho[c2];
        double Z = 0.0;
        if (c.eos == 0) Z = cs_Z(c.b_quarter * rho);
        const double divu = divergence(s_ux, s_uy, c2, W2);
        Stencil t;
        t.load(s_T, c2, W2);
        s_k1[r] = energy_rhs(c, t, s_T[c2], s_ux[c2], s_uy[c2], divu, 1.0 / rho, Z);
    }
    __syncthreads();

    // ---- phase 4: second Heun stage, collision, stores, partials ----
    Partial part = {0.0, 0.0, 0.0, 1e300, 0u};
    for (int r = tid; r < TY * TX; r += kThreads) {
        const int ry = r / TX, rx = r - ry * TX;
        const int gx = x0 + rx, gy = y0 + ry;
        if (gx >= nx || gy >= ny) continue;
        const int c2 = (ry + 2) * W2 + (rx + 2);
        const int c1 = (ry + 1) * W1 + (rx + 1);
        const int c3 = (ry + 3) * W3 + (rx + 3);
        const size_t g = (size_t)gy * nx + gx;
        const bool wall = WALLS && (gy == 0 || gy == ny - 1);
        const double rho = s_rho[c2], ux = s_ux[c2], uy = s_uy[c2], T = s_T[c2];
        const double eta = c.b_quarter * rho;

        // temperature
        double Tn;
        if (wall) {
            Tn = T;
        } else {
            double Z = 0.0;
            if (c.eos == 0) Z = cs_Z(eta);
            const double divu = divergence(s_ux, s_uy, c2, W2);
            // T~ = T^n + k1 at the node and its neighbours
            Stencil t, k;
            t.load(s_T, c2, W2);
            k.load(s_k1, c1, W1);
            Stencil tt;
            tt.e = t.e + k.e; tt.w = t.w + k.w; tt.n = t.n + k.n; tt.s = t.s + k.s;
            tt.ne = t.ne + k.ne; tt.nw = t.nw + k.nw; tt.sw = t.sw + k.sw; tt.se = t.se + k.se;
            const double k1 = s_k1[c1];
            const double k2 = energy_rhs(c, tt, T + k1, ux, uy, divu, 1.0 / rho, Z);
            Tn = T + 0.5 * (k1 + k2);
        }
        Tout[g] = Tn;

        // forces (again, from the LDS psi) for the collision
        double Fx = 0.0, Fy = 0.0, X = 0.0;
        const double psi0 = s_psi[c3];
        if (!wall) {
            Stencil p;
            p.load(s_psi, c3, W3);
            const double sx = (p.e - p.w) * (1.0 / 3.0) + ((p.ne + p.se) - (p.nw + p.sw)) * (1.0 / 12.0);
            const double sy = (p.n - p.s) * (1.0 / 3.0) + ((p.ne + p.nw) - (p.se + p.sw)) * (1.0 / 12.0);
            const double mg = -c.G * psi0;
            const double fg = (c.form == 2) ? -(rho - mean) * c.g : -rho * c.g;
            Fx = mg * sx;
            Fy = mg * sy + fg;
            // |F_int|^2 / psi^2 = G^2 |sum w psi c|^2
            X = c.G2 * (sx * sx + sy * sy);
        }

        double fs[9];
        if (TAU1) {
            // every rate 1: f* = f_eq(rho, u) + F', F' = M^-1 (S/2) =
            // w_i [3/2 (c - u).F + 9/2 (c.u)(c.F)] + sigma X (-8, 1, ..., 1)/36
            // w_i rho from one correctly rounded division (w_0 = 4/9, w_5 = 1/36
            // are exact power-of-two multiples of 1/9): multiplying by the
            // rounded constant 1/9 instead would bias the mass the same way at
            // every node and make it drift linearly over many steps
            const double r9 = rho / 9.0;
            const double uu = ux * ux + uy * uy;
            const double uF = ux * Fx + uy * Fy;
            const double base = 1.0 - 1.5 * uu;
            const double sx36 = c.sigma * X * (1.0 / 36.0);
            fs[0] = 4.0 * r9 * base - kW0 * 1.5 * uF - 8.0 * sx36;
            const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
            const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const double wi = (i < 5) ? kW1 : kW5;
                const double wr = (i < 5) ? r9 : 0.25 * r9;
                const double cu = cx[i] * ux + cy[i] * uy;
                const double cF = cx[i] * Fx + cy[i] * Fy;
                fs[i] = wr * (base + cu * (3.0 + 4.5 * cu)) + wi * (1.5 * (cF - uF) + 4.5 * cu * cF) + sx36;
            }
        } else {
            // general relaxation times: moments m = M f of the pulled
            // populations, relaxation toward m_eq, source (I - Lambda/2) S
            const int xm = (gx == 0) ? nx - 1 : gx - 1;
            const int xp = (gx == nx - 1) ? 0 : gx + 1;
            int ym = gy - 1, yp = gy + 1;
            if (!WALLS) {
                ym = (gy == 0) ? ny - 1 : ym;
                yp = (gy == ny - 1) ? 0 : yp;
            }
            const bool bot = WALLS && gy == 0, top = WALLS && gy == ny - 1;
            const size_t row = (size_t)gy * nx;
            const size_t rowm = (size_t)(bot ? gy : ym) * nx;
            const size_t rowp = (size_t)(top ? gy : yp) * nx;
            double f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            f[0] = PopIO<S>::load(fin, 0 * N + row + gx, kW0 * rr);
            f[1] = PopIO<S>::load(fin, 1 * N + row + xm, kW1 * rr);
            f[3] = PopIO<S>::load(fin, 3 * N + row + xp, kW1 * rr);
            if (!bot) {
                f[2] = PopIO<S>::load(fin, 2 * N + rowm + gx, kW1 * rr);
                f[5] = PopIO<S>::load(fin, 5 * N + rowm + xm, kW5 * rr);
                f[6] = PopIO<S>::load(fin, 6 * N + rowm + xp, kW5 * rr);
            }
            if (!top) {
                f[4] = PopIO<S>::load(fin, 4 * N + rowp + gx, kW1 * rr);
                f[7] = PopIO<S>::load(fin, 7 * N + rowp + xp, kW5 * rr);
                f[8] = PopIO<S>::load(fin, 8 * N + rowp + xm, kW5 * rr);
            }
            if (bot) {
                const double d = f[1] - f[3];
                f[2] = f[4];
                f[5] = f[7] - 0.5 * d;
                f[6] = f[8] + 0.5 * d;
            }
            if (top) {
                const double d = f[1] - f[3];
                f[4] = f[2];
                f[7] = f[5] + 0.5 * d;
                f[8] = f[6] - 0.5 * d;
            }
            // m = M f (Eq. MatrixMRT)
            const double a1 = f[1] + f[2] + f[3] + f[4];
            const double a5 = f[5] + f[6] + f[7] + f[8];
            double m[9];
            m[0] = f[0] + a1 + a5;
            m[1] = -4.0 * f[0] - a1 + 2.0 * a5;
            m[2] = 4.0 * f[0] - 2.0 * a1 + a5;
            m[3] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
            m[4] = -2.0 * (f[1] - f[3]) + f[5] - f[6] - f[7] + f[8];
            m[5] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
            m[6] = -2.0 * (f[2] - f[4]) + f[5] + f[6] - f[7] - f[8];
            m[7] = f[1] - f[2] + f[3] - f[4];
            m[8] = f[5] - f[6] + f[7] - f[8];
            // m_eq = M f_eq for the second-order equilibrium
            const double uu = ux * ux + uy * uy;
            double me[9];
            me[0] = m[0];  // mass is a collision invariant
            me[1] = rho * (-2.0 + 3.0 * uu);
            me[2] = rho * (1.0 - 3.0 * uu);
            me[3] = rho * ux;
            me[4] = -rho * ux;
            me[5] = rho * uy;
            me[6] = -rho * uy;
            me[7] = rho * (ux * ux - uy * uy);
            me[8] = rho * ux * uy;
            // (I - Lambda/2) S with S of Eq. LiFS; the sigma part reduces to
            // +sigma X/tau_e and -sigma X/tau_varsigma
            const double uF = ux * Fx + uy * Fy;
            double s[9];
            s[0] = 0.0;
            s[1] = (1.0 - 0.5 * c.lam[1]) * 6.0 * uF + c.sig_e * X;
            s[2] = -(1.0 - 0.5 * c.lam[2]) * 6.0 * uF - c.sig_s * X;
            s[3] = (1.0 - 0.5 * c.lam[3]) * Fx;
            s[4] = -(1.0 - 0.5 * c.lam[4]) * Fx;
            s[5] = (1.0 - 0.5 * c.lam[5]) * Fy;
            s[6] = -(1.0 - 0.5 * c.lam[6]) * Fy;
            s[7] = (1.0 - 0.5 * c.lam[7]) * 2.0 * (ux * Fx - uy * Fy);
            s[8] = (1.0 - 0.5 * c.lam[8]) * (ux * Fy + uy * Fx);
            double ms[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) ms[k] = m[k] - c.lam[k] * (m[k] - me[k]) + s[k];
            // f* = M^-1 m*, with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
            const double d0 = ms[0] / 9.0, d1 = ms[1] * (1.0 / 36.0), d2 = ms[2] * (1.0 / 36.0);
            const double d3 = ms[3] * (1.0 / 6.0), d4 = ms[4] * (1.0 / 12.0);
            const double d5 = ms[5] * (1.0 / 6.0), d6 = ms[6] * (1.0 / 12.0);
            const double d7 = ms[7] * 0.25, d8 = ms[8] * 0.25;
            fs[0] = d0 - 4.0 * d1 + 4.0 * d2;
            fs[1] = d0 - d1 - 2.0 * d2 + d3 - 2.0 * d4 + d7;
            fs[2] = d0 - d1 - 2.0 * d2 + d5 - 2.0 * d6 - d7;
            fs[3] = d0 - d1 - 2.0 * d2 - d3 + 2.0 * d4 + d7;
            fs[4] = d0 - d1 - 2.0 * d2 - d5 + 2.0 * d6 - d7;
            fs[5] = d0 + 2.0 * d1 + d2 + d3 + d4 + d5 + d6 + d8;
            fs[6] = d0 + 2.0 * d1 + d2 - d3 - d4 + d5 + d6 - d8;
            fs[7] = d0 + 2.0 * d1 + d2 - d3 - d4 - d5 - d6 + d8;
            fs[8] = d0 + 2.0 * d1 + d2 + d3 + d4 - d5 - d6 - d8;
        }

        // stores and the next level's mass: a population moving toward a
        // wall layer is counted twice by that wall's reconstruction; one
        // leaving through a wall is not counted
        double nm = 0.0;
        const double wr[9] = {kW0, kW1, kW1, kW1, kW1, kW5, kW5, kW5, kW5};
        const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double v = PopIO<S>::store(fout, (size_t)i * N + g, fs[i], wr[i] * rr);
            double mult = 1.0;
            if (WALLS) {
                const int yd = gy + cy[i];
                if (yd < 0 || yd >= ny)
                    mult = 0.0;
                else if ((yd == 0 && cy[i] == -1) || (yd == ny - 1 && cy[i] == 1))
                    mult = 2.0;
            }
            nm += mult * v;
        }
        part.mass_n += rho;
        part.mass_next += nm;
        part.umax = fmax(part.umax, sqrt(ux * ux + uy * uy));
        part.rmin = fmin(part.rmin, rho);
        unsigned fl = 0u;
        if (!(rho > 0.0)) fl |= kFlagRho;
        if (c.eos == 0 && eta >= 1.0) fl |= kFlagEta;
        if (psi0 != psi0) fl |= kFlagPsi;
        if (rho != rho || ux != ux || uy != uy || Tn != Tn || nm != nm) fl |= kFlagNaN;
        part.flags |= fl;
    }
    part = block_reduce<kThreads>(part, s_red, s_ured);
    finish_launch<kThreads>(part, partials, st, step, (int)((step + 1) & 1),
                            1.0 / (double)N, s_red, s_ured);
}

// ---------------------------------------------------------------------------
// Readout (off the hot loop): level-n fields from the current buffer.
// Kernel A: rho, psi, j per node into scratch; kernel B: forces, u, p_EOS and
// the normal pressure with plain central differences (interior nodes).
// ---------------------------------------------------------------------------
template <class S, bool WALLS>
__global__ void d2q9_readout_a(const S *__restrict__ fin, const double *__restrict__ Tin, Phys c,
                               int nx, int ny, double *__restrict__ scr /* 4N */)
{
    const size_t N = (size_t)nx * ny;
    const double rr = c.rho_ref;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < N;
         g += (size_t)gridDim.x * blockDim.x) {
        const int gy = (int)(g / nx), gx = (int)(g - (size_t)gy * nx);
        const int xm = (gx == 0) ? nx - 1 : gx - 1;
        const int xp = (gx == nx - 1) ? 0 : gx + 1;
        int ym = gy - 1, yp = gy + 1;
        if (!WALLS) {
            ym = (gy == 0) ? ny - 1 : ym;
            yp = (gy == ny - 1) ? 0 : yp;
        }
        const bool bot = WALLS && gy == 0, top = WALLS && gy == ny - 1;
        const size_t row = (size_t)gy * nx;
        const size_t rowm = (size_t)(bot ? gy : ym) * nx;
        const size_t rowp = (size_t)(top ? gy : yp) * nx;
        double f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        f[0] = PopIO<S>::load(fin, 0 * N + row + gx, kW0 * rr);
        f[1] = PopIO<S>::load(fin, 1 * N + row + xm, kW1 * rr);
        f[3] = PopIO<S>::load(fin, 3 * N + row + xp, kW1 * rr);
        if (!bot) {
            f[2] = PopIO<S>::load(fin, 2 * N + rowm + gx, kW1 * rr);
            f[5] = PopIO<S>::load(fin, 5 * N + rowm + xm, kW5 * rr);
            f[6] = PopIO<S>::load(fin, 6 * N + rowm + xp, kW5 * rr);
        }
        if (!top) {
            f[4] = PopIO<S>::load(fin, 4 * N + rowp + gx, kW1 * rr);
            f[7] = PopIO<S>::load(fin, 7 * N + rowp + xp, kW5 * rr);
            f[8] = PopIO<S>::load(fin, 8 * N + rowp + xm, kW5 * rr);
        }
        if (bot) {
            const double d = f[1] - f[3];
            f[2] = f[4]; f[5] = f[7] - 0.5 * d; f[6] = f[8] + 0.5 * d;
        }
        if (top) {
            const double d = f[1] - f[3];
            f[4] = f[2]; f[7] = f[5] + 0.5 * d; f[8] = f[6] - 0.5 * d;
        }
        const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        double Z;
        scr[g] = rho;
        scr[N + g] = psi_and_Z(c, rho, Tin[g], Z);
        scr[2 * N + g] = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
        scr[3 * N + g] = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    }
}

template <bool WALLS>
__global__ void d2q9_readout_b(const double *__restrict__ scr, const double *__restrict__ Tin,
                               Phys c, int nx, int ny, const StepState *__restrict__ st,
                               int slot, int field, double *__restrict__ out)
{
    const size_t N = (size_t)nx * ny;
    const double mean = st->mean[slot];
    const double *rho = scr, *psi = scr + N, *jx = scr + 2 * N, *jy = scr + 3 * N;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < N;
         g += (size_t)gridDim.x * blockDim.x) {
        const int gy = (int)(g / nx), gx = (int)(g - (size_t)gy * nx);
        const int xm = (gx == 0) ? nx - 1 : gx - 1, xp = (gx == nx - 1) ? 0 : gx + 1;
        const int ym = (gy == 0) ? ny - 1 : gy - 1, yp = (gy == ny - 1) ? 0 : gy + 1;
        const bool wall = WALLS && (gy == 0 || gy == ny - 1);
        const double r = rho[g];
        double v = 0.0;
        if (field == 4) {
            v = Tin[g];
        } else if (field == 0) {
            v = r;
        } else if (field == 5) {
            v = p_eos(c, r, Tin[g]);
        } else if (field == 6) {
            const double pe = p_eos(c, r, Tin[g]);
            if (wall) {
                v = pe;
            } else {
                const double p0 = psi[g];
                const double pE = psi[(size_t)gy * nx + xp], pW = psi[(size_t)gy * nx + xm];
                const double pN = psi[(size_t)yp * nx + gx], pS = psi[(size_t)ym * nx + gx];
                const double dx = 0.5 * (pE - pW), dy = 0.5 * (pN - pS);
                const double lap = (pE + pW) + (pN + pS) - 4.0 * p0;
                const double dyy = (pN + pS) - 2.0 * p0;
                v = pe + c.sigma * c.G2 * (1.0 / 6.0) * (dx * dx + dy * dy) +
                    c.G * (1.0 / 12.0) * p0 * lap + c.G * (1.0 / 6.0) * p0 * dyy;
            }
        } else {  // velocity components
            double Fx = 0.0, Fy = 0.0;
            if (!wall) {
                const double p0 = psi[g];
                const double pE = psi[(size_t)gy * nx + xp], pW = psi[(size_t)gy * nx + xm];
                const double pN = psi[(size_t)yp * nx + gx], pS = psi[(size_t)ym * nx + gx];
                const double pNE = psi[(size_t)yp * nx + xp], pNW = psi[(size_t)yp * nx + xm];
                const double pSW = psi[(size_t)ym * nx + xm], pSE = psi[(size_t)ym * nx + xp];
                const double sx = (pE - pW) * (1.0 / 3.0) + ((pNE + pSE) - (pNW + pSW)) * (1.0 / 12.0);
                const double sy = (pN - pS) * (1.0 / 3.0) + ((pNE + pNW) - (pSE + pSW)) * (1.0 / 12.0);
                const double fg = (c.form == 2) ? -(r - mean) * c.g : -r * c.g;
                Fx = -c.G * p0 * sx;
                Fy = -c.G * p0 * sy + fg;
            }
            if (field == 1) v = (jx[g] + 0.5 * Fx) / r;
            else if (field == 2) v = (jy[g] + 0.5 * Fy) / r;
            else v = 0.0;
        }
        out[g] = v;
    }
}

template <class S, bool TAU1, bool WALLS, int TX, int TY>
hipError_t launch_t(const LatticeLaunch &L)
{
    const int tiles_x = (L.nx + TX - 1) / TX, tiles_y = (L.ny + TY - 1) / TY;
    const int nb = tiles_x * tiles_y;
    hipLaunchKernelGGL((d2q9_step<S, TAU1, WALLS, TX, TY>), dim3(nb), dim3(kThreads), 0, L.stream,
                       (const S *)L.fin, (S *)L.fout, L.Tin, L.Tout, L.phys, L.nx, L.ny, tiles_x,
                       L.partials, L.st, L.step);
    return hipGetLastError();
}

template <class S, bool TAU1, bool WALLS>
hipError_t launch_tile(const LatticeLaunch &L)
{
    switch (L.tile) {
    case 1: return launch_t<S, TAU1, WALLS, 32, 32>(L);
    case 2: return launch_t<S, TAU1, WALLS, 128, 8>(L);
    default: return launch_t<S, TAU1, WALLS, 64, 16>(L);
    }
}

}  // namespace

int d2q9_num_blocks(int nx, int ny, int tile)
{
    int TX = 64, TY = 16;
    if (tile == 1) { TX = 32; TY = 32; }
    if (tile == 2) { TX = 128; TY = 8; }
    return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
}

hipError_t d2q9_launch_step(const LatticeLaunch &L)
{
    if (L.fp32) {
        if (L.tau1) return L.walls ? launch_tile<float, true, true>(L) : launch_tile<float, true, false>(L);
        return L.walls ? launch_tile<float, false, true>(L) : launch_tile<float, false, false>(L);
    }
    if (L.tau1) return L.walls ? launch_tile<double, true, true>(L) : launch_tile<double, true, false>(L);
    return L.walls ? launch_tile<double, false, true>(L) : launch_tile<double, false, false>(L);
}

hipError_t d2q9_launch_readout(const LatticeLaunch &L, int field, double *scratch, double *out)
{
    const size_t N = (size_t)L.nx * L.ny;
    const int threads = 256;
    const int blocks = (int)((N + threads - 1) / threads < 65535 ? (N + threads - 1) / threads : 65535);
    if (L.fp32) {
        if (L.walls)
            hipLaunchKernelGGL((d2q9_readout_a<float, true>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const float *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch);
        else
            hipLaunchKernelGGL((d2q9_readout_a<float, false>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const float *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch);
    } else {
        if (L.walls)
            hipLaunchKernelGGL((d2q9_readout_a<double, true>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const double *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch);
        else
            hipLaunchKernelGGL((d2q9_readout_a<double, false>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const double *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.walls)
        hipLaunchKernelGGL((d2q9_readout_b<true>), dim3(blocks), dim3(threads), 0, L.stream, scratch,
                           L.Tin, L.phys, L.nx, L.ny, L.st, (int)(L.step & 1), field, out);
    else
        hipLaunchKernelGGL((d2q9_readout_b<false>), dim3(blocks), dim3(threads), 0, L.stream, scratch,
                           L.Tin, L.phys, L.nx, L.ny, L.st, (int)(L.step & 1), field, out);
    return hipGetLastError();
}

}  // namespace tplbm
