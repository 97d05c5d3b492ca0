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
//
// Launch shape: a persistent grid of one 1024-thread block per compute unit;
// the blocks of each XCD walk a contiguous range of 64 x 32 tiles, so the
// halo rows that neighbouring tiles share are served by that XCD's L2.
#include <hip/hip_runtime.h>

#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {


template <class S>
struct PopIO;
template <>
struct PopIO<double> {
    __device__ static __forceinline__ double load(const double *p, size_t i, double /*wref*/)
    {
        return p[i];
    }
    template <bool STREAM>
    __device__ static __forceinline__ double store(double *p, size_t i, double v, double)
    {
        if (STREAM) __builtin_nontemporal_store(v, &p[i]);
        else p[i] = v;
        return v;
    }
};
template <>
struct PopIO<float> {
    // FP32 deviation storage: the stored value is f_i - w_i rho_ref(layer),
    // with the reference density of the layer (row) the value is stored in
    __device__ static __forceinline__ double load(const float *p, size_t i, double wref)
    {
        return wref + (double)p[i];
    }
    template <bool STREAM>
    __device__ static __forceinline__ double store(float *p, size_t i, double v, double wref)
    {
        const float d = (float)(v - wref);
        if (STREAM) __builtin_nontemporal_store(d, &p[i]);
        else p[i] = d;
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
    // gradient and 6 sum_i w_i (phi_i - phi_0) together.  The Laplacian sums
    // equal neighbours pairwise before subtracting 4 phi_0, so it vanishes
    // exactly on a uniform field (2 phi and 4 phi are exact).
    __device__ __forceinline__ void grad_lap(double c0, double &gx, double &gy, double &lap) const
    {
        const double a = ne + se, b = nw + sw, p = ne + nw, q = se + sw;
        gx = (e - w) * (1.0 / 3.0) + (a - b) * (1.0 / 12.0);
        gy = (n - s) * (1.0 / 3.0) + (p - q) * (1.0 / 12.0);
        const double c4 = 4.0 * c0;
        lap = (((e + w) + (n + s)) - c4) * (2.0 / 3.0) + ((a + b) - c4) * (1.0 / 6.0);
    }
};

// Right-hand side of the energy equation at one node, for the field whose
// stencil values are in t and centre value is T0.
__device__ __forceinline__ double energy_rhs(const Phys &c, const Stencil &t, double T0, double ux,
                                             double uy, double divu, double inv_rho, double Z)
{
    double gx, gy, lap;
    t.grad_lap(T0, gx, gy, lap);
    const double adv = -(ux * gx + uy * gy);
    const double cond = c.kappa_over_cv * inv_rho * lap;
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

// Zou-He reconstruction (zero wall velocity) of the populations a wall node
// does not receive, then density and momentum of the pulled set.
__device__ __forceinline__ void pulled_moments(double f[9], bool bot, bool top, double &rho, double &jx,
                                               double &jy)
{
    if (bot) {  // unknowns 2, 5, 6
        const double d = f[1] - f[3];
        f[2] = f[4];
        f[5] = f[7] - 0.5 * d;
        f[6] = f[8] + 0.5 * d;
    }
    if (top) {  // unknowns 4, 7, 8
        const double d = f[1] - f[3];
        f[4] = f[2];
        f[7] = f[5] + 0.5 * d;
        f[8] = f[6] - 0.5 * d;
    }
    rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
}

// Shan-Chen force on the psi stencil (LDS, centre index c3, row stride ld)
// plus gravity (sub: the density the gravity form subtracts), and
// X = |F_int|^2 / psi^2 = G^2 |sum w psi c|^2 for the sigma
// term.  Zero at wall nodes.
__device__ __forceinline__ void node_force(const Phys &c, const double *s_psi, int c3, int ld, double rho,
                                           double sub, bool wall, double &Fx, double &Fy, double &X)
{
    Fx = Fy = X = 0.0;
    if (wall) return;
    Stencil p;
    p.load(s_psi, c3, ld);
    const double sx = (p.e - p.w) * (1.0 / 3.0) + ((p.ne + p.se) - (p.nw + p.sw)) * (1.0 / 12.0);
    const double sy = (p.n - p.s) * (1.0 / 3.0) + ((p.ne + p.nw) - (p.se + p.sw)) * (1.0 / 12.0);
    const double mg = -c.G * s_psi[c3];
    const double fg = gravity_force(rho, sub, c.g);
    Fx = mg * sx;
    Fy = mg * sy + fg;
    X = c.G2 * (sx * sx + sy * sy);
}

// Every relaxation rate 1: f* = f_eq(rho, u) + F', F' = M^-1 (S/2) =
// w_i [3/2 (c - u).F + 9/2 (c.u)(c.F)] + sigma X (-8, 1, ..., 1)/36.  The
// rest population is closed by mass conservation, f*_0 = rho - sum_{i>0}
// f*_i (exact in exact arithmetic), so the collision adds no systematic
// rounding drift to the mass.  Opposite velocities share the even part of
// f_eq + F' and differ in the sign of the odd part: per pair (i, i')
// f*_i = E + O, f*_i' = E - O with
// E = w rho (1 - 3/2 u^2 + 9/2 (c.u)^2) + w (9/2 (c.u)(c.F) - 3/2 u.F) + sigma X/36
// O = w (3 rho c.u + 3/2 c.F)
__device__ __forceinline__ void collide_tau1(const Phys &c, double rho, double ux, double uy, double Fx,
                                             double Fy, double X, double fs[9])
{
    const double uu = ux * ux + uy * uy;
    const double uF = ux * Fx + uy * Fy;
    const double sx36 = c.sigma * X * (1.0 / 36.0);
    const double r1 = kW1 * rho, r5 = kW5 * rho;
    const double b1 = r1 * (1.0 - 1.5 * uu) - kW1 * 1.5 * uF + sx36;
    const double b5 = r5 * (1.0 - 1.5 * uu) - kW5 * 1.5 * uF + sx36;
    auto pair = [&](double cu, double cF, double wr, double wi, double base, double &fp, double &fm) {
        const double E = base + 4.5 * cu * (wr * cu + wi * cF);
        const double O = 3.0 * wr * cu + 1.5 * wi * cF;
        fp = E + O;
        fm = E - O;
    };
    pair(ux, Fx, r1, kW1, b1, fs[1], fs[3]);
    pair(uy, Fy, r1, kW1, b1, fs[2], fs[4]);
    pair(ux + uy, Fx + Fy, r5, kW5, b5, fs[5], fs[7]);
    pair(uy - ux, Fy - Fx, r5, kW5, b5, fs[6], fs[8]);
    const double rest = ((fs[1] + fs[2]) + (fs[3] + fs[4])) + ((fs[5] + fs[6]) + (fs[7] + fs[8]));
    fs[0] = rho - rest;
}

// Next level's mass contribution of a node's post-collision set: a
// population moving into a wall layer is counted twice by that wall's
// reconstruction; one leaving through a wall is not counted.
template <bool WALLS>
__device__ __forceinline__ double next_mass(const double v[9], int gy, int ny)
{
    double nm = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])) + v[8];
    if (WALLS) {
        const double down = (v[4] + v[7]) + v[8], up = (v[2] + v[5]) + v[6];
        if (gy == 0) nm -= down;
        if (gy == 1) nm += down;
        if (gy == ny - 2) nm += up;
        if (gy == ny - 1) nm -= up;
    }
    return nm;
}

// Register-resident pulled populations of the region nodes one thread owns
// in phase 1 (raw stored values; converted when consumed).  All of them are
// loaded before the first is used, so a tile costs one memory round trip.
template <class S, int NSLOT>
struct Prefetch {
    S f[NSLOT][9];
    double T[NSLOT];
};

// Geometry of one region node: global coordinates and the flat indices of
// its own node and of the three rows the pull reads.  Rows beyond a wall are
// clamped to the node's own row (those populations are reconstructed, never
// used as loaded); nodes beyond a wall are clamped in-bounds and flagged.
struct NodeGeom {
    int gx, gy;
    bool valid, bot, top;
    unsigned row, rowm, rowp, xm, xp;
};

template <bool WALLS, int W3, int TY>
__device__ __forceinline__ NodeGeom region_node(int r, int x0, int y0, int nx, int ny, bool small_x)
{
    NodeGeom q;
    const int ry = r / W3, rx = r - ry * W3;
    int gx = x0 + rx - 3;
    if (small_x) {
        gx %= nx;
        if (gx < 0) gx += nx;
    } else {
        gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    }
    int gy = y0 + ry - 3;
    q.valid = true;
    if (WALLS) {
        q.valid = (gy >= 0 && gy < ny);
        gy = gy < 0 ? 0 : (gy >= ny ? ny - 1 : gy);
        q.bot = q.valid && gy == 0;
        q.top = q.valid && gy == ny - 1;
        q.rowm = (unsigned)(gy == 0 ? gy : gy - 1) * (unsigned)nx;
        q.rowp = (unsigned)(gy == ny - 1 ? gy : gy + 1) * (unsigned)nx;
    } else {
        if (small_x || ny < TY + 6) {  // tiny lattices: general wrap
            gy %= ny;
            if (gy < 0) gy += ny;
        } else {
            gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
        }
        q.bot = q.top = false;
        q.rowm = (unsigned)(gy == 0 ? ny - 1 : gy - 1) * (unsigned)nx;
        q.rowp = (unsigned)(gy == ny - 1 ? 0 : gy + 1) * (unsigned)nx;
    }
    q.gx = gx;
    q.gy = gy;
    q.row = (unsigned)gy * (unsigned)nx;
    q.xm = (unsigned)(gx == 0 ? nx - 1 : gx - 1);
    q.xp = (unsigned)(gx == nx - 1 ? 0 : gx + 1);
    return q;
}

// Reference terms w_i rho_ref(layer of the stored value) of a node's pulled
// set: directions 0, 1, 3 come from its own row, 2, 5, 6 from the row below,
// 4, 7, 8 from the row above.  `lr` holds the references of consecutive rows
// and `k` is the index of the node's own row in it.  FP64 storage has no
// reference.
template <class S>
__device__ __forceinline__ void pull_refs(const double *lr, int k, double (&w)[9])
{
    if (sizeof(S) == 8) {
#pragma unroll
        for (int i = 0; i < 9; ++i) w[i] = 0.0;
        return;
    }
    const double r0 = lr[k], rm = lr[k - 1], rp = lr[k + 1];
    w[0] = kW0 * r0;
    w[1] = kW1 * r0;
    w[3] = kW1 * r0;
    w[2] = kW1 * rm;
    w[5] = kW5 * rm;
    w[6] = kW5 * rm;
    w[4] = kW1 * rp;
    w[7] = kW5 * rp;
    w[8] = kW5 * rp;
}

// Issue the pull loads [i0, i1) of one region node (all in-bounds); loads
// 0..8 are the populations, load 9 the temperature.
template <class S>
__device__ __forceinline__ void pull_loads(const S *__restrict__ fin, const double *__restrict__ Tin,
                                           size_t N, const NodeGeom &q, S (&f)[9], double &T, int i0 = 0,
                                           int i1 = 10)
{
    const unsigned gx = (unsigned)q.gx;
    const unsigned idx[9] = {q.row + gx, q.row + q.xm, q.rowm + gx, q.row + q.xp, q.rowp + gx,
                             q.rowm + q.xm, q.rowm + q.xp, q.rowp + q.xp, q.rowp + q.xm};
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i >= i0 && i < i1) f[i] = fin[(size_t)i * N + idx[i]];
    if (9 >= i0 && 9 < i1) T = Tin[q.row + gx];
}

template <class S, bool TAU1, bool WALLS, int TX, int TY, int NT, int MIN_WAVES_PER_EU, int PFP, bool STREAM>
__global__ __launch_bounds__(NT, MIN_WAVES_PER_EU) void d2q9_step(const S *__restrict__ fin,
                                                         S *__restrict__ fout,
                                                         const double *__restrict__ Tin,
                                                         double *__restrict__ Tout, Phys c,
                                                         int nx, int ny, int tiles_x, int ntiles,
                                                         double *__restrict__ partials,
                                                         StepState *__restrict__ st,
                                                         int64_t step,
                                                         const double *__restrict__ rref)
{
    constexpr int kThreads = NT;
    constexpr int W3 = TX + 6, H3 = TY + 6;
    constexpr int W2 = TX + 4, H2 = TY + 4;
    constexpr int W1 = TX + 2, H1 = TY + 2;
    constexpr int R3N = H3 * W3;
    constexpr int NSLOT = (R3N + kThreads - 1) / kThreads;
    __shared__ double s_psi[R3N];
    __shared__ double s_rho[H2 * W2];
    __shared__ double s_T[H2 * W2];
    __shared__ double s_ux[H2 * W2];
    __shared__ double s_uy[H2 * W2];
    __shared__ double s_Z[H2 * W2];
    __shared__ double s_k1[H1 * W1];   // first Heun stage K(T^n); T~ = T^n + k1
    __shared__ double s_div[H1 * W1];  // div u, for both Heun stages
    __shared__ double s_red[4 * kThreads / 64];
    __shared__ unsigned s_ured[kThreads / 64];
    // FP32 deviations: row references of a tile's region rows and the rows
    // its pulls reach, y0 - 4 .. y0 + TY + 3 (rows beyond a wall are clamped:
    // the populations pulled from there are reconstructed, never used);
    // double-buffered so that the next tile's rows load during this tile
    constexpr int NR = TY + 8;
    __shared__ double s_rref[2][NR];

    const int tid = threadIdx.x;
    const size_t N = (size_t)nx * ny;
    const double mean = st->mean[step & 1];
    const double sub = gravity_sub(c.form, mean, c.rho_v);
    const bool small_x = nx < W3;
    auto ref_row = [&](int y) {
        if (WALLS) return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        return wrapi(y, ny);
    };

    // Tiles of this block: blocks are dispatched round-robin over the 8 XCDs;
    // each XCD gets a contiguous range of tiles so that halos are shared in
    // its L2, and the blocks of one XCD stride through that range.
    const int nb = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per_xcd_blocks = nb >> 3;  // nb is a multiple of 8
    const int tiles_per_xcd = (ntiles + 7) >> 3;
    const int t_begin = xcd * tiles_per_xcd;
    const int t_end = min(ntiles, t_begin + tiles_per_xcd);

    Prefetch<S, NSLOT> pre;
    // issue loads [i0, i1) of the first region slot of tile t (early), or the
    // remaining loads of the tile
    auto issue = [&](int t, bool early) {
        const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
#pragma unroll
        for (int k = 0; k < NSLOT; ++k) {
            const int r = tid + k * kThreads;
            const int i0 = early ? 0 : (k == 0 ? PFP : 0);
            const int i1 = early ? (k == 0 ? PFP : 0) : 10;
            if (i0 < i1 && r < R3N) {
                const NodeGeom q = region_node<WALLS, W3, TY>(r, x0, y0, nx, ny, small_x);
                pull_loads<S>(fin, Tin, N, q, pre.f[k], pre.T[k], i0, i1);
            }
        }
    };

    Partial part = {0.0, 0.0, 0.0, 1e300, 0u};
    // The first PFP loads of a tile's first region slot are issued during the
    // previous tile's last phase (that slot is consumed first), the rest at
    // the start of the tile: every pull is issued before any is consumed, and
    // part of them is in flight while the previous tile computes.
    if (t_begin + slot < t_end) issue(t_begin + slot, true);
    if (sizeof(S) == 4) {
        if (tid < NR && t_begin + slot < t_end)
            s_rref[0][tid] = rref[ref_row(((t_begin + slot) / tiles_x) * TY - 4 + tid)];
        __syncthreads();
    }
    int rb = 0;  // buffer of s_rref holding this tile's rows
    for (int t = t_begin + slot; t < t_end; t += per_xcd_blocks, rb ^= 1) {
        const int x0 = (t % tiles_x) * TX, y0 = (t / tiles_x) * TY;
        issue(t, false);
        const double *lref = s_rref[rb];

        // ---- phase 1: density, momentum, psi on tile + 3 (from registers) ----
#pragma unroll
        for (int k = 0; k < NSLOT; ++k) {
            const int r = tid + k * kThreads;
            if (r < R3N) {
                const NodeGeom q = region_node<WALLS, W3, TY>(r, x0, y0, nx, ny, small_x);
                double wref[9], f[9];
                pull_refs<S>(lref, r / W3 + 1, wref);  // region row ry is y0 + ry - 3
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = PopIO<S>::load(pre.f[k], i, wref[i]);
                double rho, jx, jy;
                pulled_moments(f, WALLS && q.bot, WALLS && q.top, rho, jx, jy);
                double Z = 0.0, psi = 0.0, T = pre.T[k];
                if (q.valid) {
                    psi = psi_and_Z(c, rho, T, Z);
                } else {
                    rho = jx = jy = T = 0.0;
                }
                s_psi[r] = psi;
                const int ry = r / W3, rx = r - ry * W3;
                if (rx >= 1 && rx < W3 - 1 && ry >= 1 && ry < H3 - 1) {
                    const int qi = (ry - 1) * W2 + (rx - 1);
                    s_rho[qi] = rho;
                    s_T[qi] = T;
                    s_ux[qi] = jx;
                    s_uy[qi] = jy;
                    s_Z[qi] = Z;
                }
            }
        }
        __syncthreads();

        // ---- phase 2: force and force-corrected velocity on tile + 2 ----
        for (int r = tid; r < H2 * W2; r += kThreads) {
            const int ry = r / W2, rx = r - ry * W2;
            const int gy = y0 + ry - 2;
            bool valid = true, wall = false;
            if (WALLS) {
                valid = (gy >= 0 && gy < ny);
                wall = (gy == 0 || gy == ny - 1);
            }
            if (!valid) continue;
            const double rho = s_rho[r];
            double Fx, Fy, X;
            node_force(c, s_psi, (ry + 1) * W3 + (rx + 1), W3, rho, sub, wall, Fx, Fy, X);
            const double inv = rcp_pos(rho);
            s_ux[r] = (s_ux[r] + 0.5 * Fx) * inv;
            s_uy[r] = (s_uy[r] + 0.5 * Fy) * inv;
        }
        __syncthreads();

        // ---- phase 3: first Heun stage on tile + 1 ----
        for (int r = tid; r < H1 * W1; r += kThreads) {
            const int ry = r / W1, rx = r - ry * W1;
            const int gy = y0 + ry - 1;
            const int c2 = (ry + 1) * W2 + (rx + 1);
            if (WALLS && (gy <= 0 || gy >= ny - 1)) {
                s_k1[r] = 0.0;  // Dirichlet walls (and nodes beyond them): T~ = T
                s_div[r] = 0.0;
                continue;
            }
            const double divu = divergence(s_ux, s_uy, c2, W2);
            Stencil tt;
            tt.load(s_T, c2, W2);
            s_k1[r] = energy_rhs(c, tt, s_T[c2], s_ux[c2], s_uy[c2], divu, rcp_pos(s_rho[c2]), s_Z[c2]);
            s_div[r] = divu;
        }
        __syncthreads();

        if (t + per_xcd_blocks < t_end) {
            issue(t + per_xcd_blocks, true);
            // the next tile's row references go to the other buffer (read
            // after this tile's closing barrier)
            if (sizeof(S) == 4 && tid < NR)
                s_rref[rb ^ 1][tid] = rref[ref_row(((t + per_xcd_blocks) / tiles_x) * TY - 4 + tid)];
        }

        // ---- phase 4: second Heun stage, collision, stores, partials ----
        for (int r = tid; r < TY * TX; r += kThreads) {
            const int ry = r / TX, rx = r - ry * TX;
            const int gx = x0 + rx, gy = y0 + ry;
            if (gx >= nx || gy >= ny) continue;
            const int c2 = (ry + 2) * W2 + (rx + 2);
            const int c1 = (ry + 1) * W1 + (rx + 1);
            const int c3 = (ry + 3) * W3 + (rx + 3);
            const unsigned g = (unsigned)gy * (unsigned)nx + (unsigned)gx;
            const bool wall = WALLS && (gy == 0 || gy == ny - 1);
            const double rho = s_rho[c2], ux = s_ux[c2], uy = s_uy[c2], T = s_T[c2];

            // temperature
            double Tn = T;
            if (!wall) {
                const double divu = s_div[c1];
                Stencil tt, kk;  // T~ = T^n + k1 at the node and its neighbours
                tt.load(s_T, c2, W2);
                kk.load(s_k1, c1, W1);
                tt.e += kk.e; tt.w += kk.w; tt.n += kk.n; tt.s += kk.s;
                tt.ne += kk.ne; tt.nw += kk.nw; tt.sw += kk.sw; tt.se += kk.se;
                const double k1 = s_k1[c1];
                const double k2 = energy_rhs(c, tt, T + k1, ux, uy, divu, rcp_pos(rho), s_Z[c2]);
                Tn = T + 0.5 * (k1 + k2);
            }
            Tout[g] = Tn;

            // forces (again, from the LDS psi) for the collision
            double Fx, Fy, X;
            const double psi0 = s_psi[c3];
            node_force(c, s_psi, c3, W3, rho, sub, wall, Fx, Fy, X);

            double fs[9];
            if (TAU1) {
                collide_tau1(c, rho, ux, uy, Fx, Fy, X, fs);
            } else {
                // general relaxation times: moments m = M f of the pulled
                // populations, relaxation toward m_eq, source (I - Lambda/2) S
                const NodeGeom q = region_node<WALLS, W3, TY>((ry + 3) * W3 + (rx + 3), x0, y0, nx, ny, small_x);
                S raw[9];
                double Tdummy;
                pull_loads<S>(fin, Tin, N, q, raw, Tdummy);
                double wref[9], f[9];
                pull_refs<S>(lref, ry + 4, wref);
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = PopIO<S>::load(raw, i, wref[i]);
                if (WALLS && q.bot) {
                    const double d = f[1] - f[3];
                    f[2] = f[4];
                    f[5] = f[7] - 0.5 * d;
                    f[6] = f[8] + 0.5 * d;
                }
                if (WALLS && q.top) {
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
                double sv[9];
                sv[0] = 0.0;
                sv[1] = (1.0 - 0.5 * c.lam[1]) * 6.0 * uF + c.sig_e * X;
                sv[2] = -(1.0 - 0.5 * c.lam[2]) * 6.0 * uF - c.sig_s * X;
                sv[3] = (1.0 - 0.5 * c.lam[3]) * Fx;
                sv[4] = -(1.0 - 0.5 * c.lam[4]) * Fx;
                sv[5] = (1.0 - 0.5 * c.lam[5]) * Fy;
                sv[6] = -(1.0 - 0.5 * c.lam[6]) * Fy;
                sv[7] = (1.0 - 0.5 * c.lam[7]) * 2.0 * (ux * Fx - uy * Fy);
                sv[8] = (1.0 - 0.5 * c.lam[8]) * (ux * Fy + uy * Fx);
                double ms[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) ms[k] = m[k] - c.lam[k] * (m[k] - me[k]) + sv[k];
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

            // stores (FP32: relative to this row's reference), and the next level's mass
            const double ry_ref = sizeof(S) == 4 ? lref[ry + 4] : 0.0;
            const double wst[9] = {kW0 * ry_ref, kW1 * ry_ref, kW1 * ry_ref, kW1 * ry_ref, kW1 * ry_ref,
                                   kW5 * ry_ref, kW5 * ry_ref, kW5 * ry_ref, kW5 * ry_ref};
            double v[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                v[i] = PopIO<S>::template store<STREAM>(fout, (size_t)i * N + g, fs[i], wst[i]);
            const double nm = next_mass<WALLS>(v, gy, ny);
            part.mass_n += rho;
            part.mass_next += nm;
            part.umax = fmax(part.umax, ux * ux + uy * uy);
            part.rmin = fmin(part.rmin, rho);
            unsigned fl = 0u;
            if (!(rho > 0.0)) fl |= kFlagRho;
            if (c.eos == 0 && c.b_quarter * rho >= 1.0) fl |= kFlagEta;
            if (psi0 != psi0) fl |= kFlagPsi;
            if (rho != rho || ux != ux || uy != uy || Tn != Tn || nm != nm) fl |= kFlagNaN;
            part.flags |= fl;
        }
        __syncthreads();  // LDS is rewritten by the next tile's phase 1
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
                               int nx, int ny, double *__restrict__ scr /* 4N */,
                               const double *__restrict__ rref)
{
    const size_t N = (size_t)nx * ny;
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
        // FP32: references of the rows the values are stored in
        const double r0 = sizeof(S) == 4 ? rref[gy] : 0.0;
        const double rm = sizeof(S) == 4 ? rref[bot ? gy : ym] : 0.0;
        const double rp = sizeof(S) == 4 ? rref[top ? gy : yp] : 0.0;
        double f[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        f[0] = PopIO<S>::load(fin, 0 * N + row + gx, kW0 * r0);
        f[1] = PopIO<S>::load(fin, 1 * N + row + xm, kW1 * r0);
        f[3] = PopIO<S>::load(fin, 3 * N + row + xp, kW1 * r0);
        if (!bot) {
            f[2] = PopIO<S>::load(fin, 2 * N + rowm + gx, kW1 * rm);
            f[5] = PopIO<S>::load(fin, 5 * N + rowm + xm, kW5 * rm);
            f[6] = PopIO<S>::load(fin, 6 * N + rowm + xp, kW5 * rm);
        }
        if (!top) {
            f[4] = PopIO<S>::load(fin, 4 * N + rowp + gx, kW1 * rp);
            f[7] = PopIO<S>::load(fin, 7 * N + rowp + xp, kW5 * rp);
            f[8] = PopIO<S>::load(fin, 8 * N + rowp + xm, kW5 * rp);
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

// Readout kernel A for the moment state: the level's rho and j are stored.
__global__ void d2q9_readout_a_mom(const double *__restrict__ M, const double *__restrict__ Tin, Phys c,
                                   int nx, int ny, double *__restrict__ scr /* 4N */)
{
    const size_t N = (size_t)nx * ny;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < N;
         g += (size_t)gridDim.x * blockDim.x) {
        const double rho = M[g];
        double Z;
        scr[g] = rho;
        scr[N + g] = psi_and_Z(c, rho, Tin[g], Z);
        scr[2 * N + g] = M[N + g];
        scr[3 * N + g] = M[2 * N + g];
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
                const double fg = gravity_force(r, gravity_sub(c.form, mean, c.rho_v), c.g);
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

// Tile of 64 x 32 nodes per block of 1024 threads (16 wavefronts): the LDS
// staging of a tile (about 137 KB) allows one block per compute unit.
constexpr int kTX = 64, kTY = 32, kNT = 1024;

template <class S, bool TAU1, bool WALLS>
hipError_t launch_t(const LatticeLaunch &L)
{
    const int tiles_x = (L.nx + kTX - 1) / kTX, tiles_y = (L.ny + kTY - 1) / kTY;
    const int ntiles = tiles_x * tiles_y;
    const int nb = d2q9_num_blocks(L.nx, L.ny, L.resident);
    // How many loads of the next tile's first region slot are issued before
    // the last phase of the current tile: with FP32 storage all of them
    // (populations and temperature) fit in registers; with FP64 storage the
    // first three populations do, more would spill.  The general-relaxation
    // collision needs those registers itself.
    constexpr int PFP = TAU1 ? (sizeof(S) == 4 ? 10 : 3) : 0;
    // Populations are stored with the non-temporal policy when the two levels
    // do not fit in three quarters of the 256 MiB last-level (infinity) cache:
    // the next step then reads them from HBM anyway (1024 x 2048 FP64: 94 ->
    // 87 us per step); a state that fits is re-read from that cache, and
    // streaming its stores past it measured slower (FP32: 66 -> 72 us).
    const bool stream = 2 * 9 * (size_t)L.nx * L.ny * sizeof(S) > (size_t(192) << 20);
    auto kern = stream ? d2q9_step<S, TAU1, WALLS, kTX, kTY, kNT, 4, PFP, true>
                       : d2q9_step<S, TAU1, WALLS, kTX, kTY, kNT, 4, PFP, false>;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kNT), 0, L.stream, (const S *)L.fin, (S *)L.fout, L.Tin, L.Tout, L.phys,
                       L.nx, L.ny, tiles_x, ntiles, L.partials, L.st, L.step, L.rref);
    return hipGetLastError();
}

}  // namespace

// Persistent grid of the population kernels: one block per compute unit (at
// most one per tile), a multiple of 8 so that every XCD gets the same number
// of blocks.  The moment state is updated by the row-marching kernel.
int d2q9_num_blocks(int nx, int ny, int cus, bool moments)
{
    if (moments) return d2q9_march_blocks(nx, ny, cus);
    const int ntiles = ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
    int nb = ntiles < cus ? ntiles : cus;
    nb = ((nb + 7) / 8) * 8;
    return nb;
}

hipError_t d2q9_launch_step(const LatticeLaunch &L)
{
    if (L.moments) return d2q9_march_launch(L);
    if (L.fp32) {
        if (L.tau1) return L.walls ? launch_t<float, true, true>(L) : launch_t<float, true, false>(L);
        return L.walls ? launch_t<float, false, true>(L) : launch_t<float, false, false>(L);
    }
    if (L.tau1) return L.walls ? launch_t<double, true, true>(L) : launch_t<double, true, false>(L);
    return L.walls ? launch_t<double, false, true>(L) : launch_t<double, false, false>(L);
}

hipError_t d2q9_launch_readout(const LatticeLaunch &L, int field, double *scratch, double *out)
{
    const size_t N = (size_t)L.nx * L.ny;
    const int threads = 256;
    const int blocks = (int)((N + threads - 1) / threads < 65535 ? (N + threads - 1) / threads : 65535);
    if (L.moments) {
        hipLaunchKernelGGL(d2q9_readout_a_mom, dim3(blocks), dim3(threads), 0, L.stream, (const double *)L.fin,
                           L.Tin, L.phys, L.nx, L.ny, scratch);
    } else if (L.fp32) {
        if (L.walls)
            hipLaunchKernelGGL((d2q9_readout_a<float, true>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const float *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch, L.rref);
        else
            hipLaunchKernelGGL((d2q9_readout_a<float, false>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const float *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch, L.rref);
    } else {
        if (L.walls)
            hipLaunchKernelGGL((d2q9_readout_a<double, true>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const double *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch, L.rref);
        else
            hipLaunchKernelGGL((d2q9_readout_a<double, false>), dim3(blocks), dim3(threads), 0, L.stream,
                               (const double *)L.fin, L.Tin, L.phys, L.nx, L.ny, scratch, L.rref);
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
