// D2Q9 update on the moment state (every relaxation rate 1) by row marching.
//
// One wavefront owns a strip of at most 58 columns and a range of rows (a
// segment).  Its 64 lanes hold the strip's columns plus three halo columns on
// each side: lane l is column x0 - 3 + l (periodic in x).  The wavefront
// walks the rows of its segment upwards; the step that loads row a of the
// level-n state finishes one row of every stage of the update (Sec. III):
//   row a     (rho, j) and T^n loaded; psi and Z(eta)           Eqs. EOS, InteractionPotential
//   row a - 1 Shan-Chen force, gravity, u = (j + F/2)/rho        Eqs. ShanChenForce, Gravity_*, Momentum
//   row a - 2 first Heun stage k1 = K(T^n), T~ = T^n + k1, div u Eq. Energy_Equation
//   row a - 3 second Heun stage and T^{n+1}; tau = 1 collision with Li's forcing
//   row a - 4 pull-streaming of the post-collision sets, Zou-He at the walls, (rho, j)^{n+1}
// A stage reads the rows it needs below and above from registers: every
// per-row quantity lives in a four-row ring indexed by the row modulo 4, and
// the march is unrolled four times so that every ring index is a compile-time
// constant (no copies between rows).  Neighbours across columns come from the
// adjacent lanes by DPP wavefront shifts.  Nothing goes through LDS and the
// march takes no barrier; each stencil is evaluated once per node.
//
// A row of a stencil field is kept as its value c, the difference of its
// right and left neighbours d and their sum s.  The isotropic gradient and
// Laplacian of a node (weights w_i / c_s^2 of the D2Q9 set) follow from the
// rows below (m), at (0) and above (p):
//   d/dx = d0/3 + (dp + dm)/12,   d/dy = (cp - cm)/3 + (sp - sm)/12,
//   lap  = ((s0 + (cp + cm)) - 4 c0) 2/3 + ((sp + sm) - 4 c0)/6,
// where pairs of equal neighbours are summed before 4 c0 is subtracted, so
// the Laplacian of a uniform field is exactly zero.
//
// Rows below the first and above the last row of a lattice with walls hold
// zeros (no state there); the wall rows themselves carry no force, keep
// their temperature and receive the Zou-He reconstruction.  Without walls
// the rows wrap.  Per-lane diagnostics (mass of level n and of the next
// level, max |u|^2, min rho, flags) are reduced over the block and the grid
// as in the tile kernels.
#include <hip/hip_runtime.h>

#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {

constexpr int kHalo = 3;
constexpr int kStrip = 64 - 2 * kHalo;  // interior columns of a wavefront
constexpr int kNT = 256;                // four independent wavefronts per block
constexpr int kPF = 2;                  // rows of loads in flight ahead of use
static_assert(kPF >= 2 && kPF <= 3, "a load slot must be free when its row is issued");
constexpr double kW1 = 1.0 / 9.0, kW5 = 1.0 / 36.0;

// lane l receives the value of lane l - 1 (the column to its left; lane 0
// receives zero)
__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// lane l receives the value of lane l + 1 (the column to its right; lane 63
// receives zero)
__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Row accesses go through buffer resources whose range is one row of one
// plane: a lane outside the range (a halo lane's store, every lane of a row
// the march does not need) reads zero and writes nothing.  This keeps every
// load and store out of branches, so the compiler's wait counts for the
// loads in flight stay exact.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dword access (gfx9 family)
constexpr unsigned kOut = 0x80000000u;  // a byte offset beyond every row's range

__device__ __forceinline__ double row_load(const double *row, int bytes, unsigned off)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, bytes, kRsrcWord3);
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

__device__ __forceinline__ void row_store(double *row, int bytes, unsigned off, double v)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, bytes, kRsrcWord3);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// sqrt_pos without a branch: the same refined reciprocal square root for a
// positive argument, zero for zero, NaN for a negative or NaN argument.
__device__ __forceinline__ double sqrt_pos_sel(double a)
{
    const bool pos = a > 0.0;
    const double x = pos ? a : 1.0;
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    const double s = fma(d, h, g);
    return pos ? s : (a == 0.0 ? 0.0 : __builtin_nan(""));
}

// Per-row quantities of one lane, four rows each (index: row & 3 relative
// to the segment's first row).
struct Rings {
    double pc[4], pd[4], ps[4];                 // psi
    double rho[4], jx[4], jy[4], Z[4];
    double tc[4], td[4], ts[4];                 // T^n
    double ux[4], uy[4], uxd[4], uys[4], inv[4];
    double ttc[4], ttd[4], tts[4], k1[4], dv[4];  // T~ = T^n + k1, k1, div u
    double pull[4][9];                          // pulled sets being assembled
    double lr[4], ljx[4], ljy[4], lT[4];        // loads in flight
    double mass_n, mass_next, umax, rmin;       // diagnostics of the lane's own nodes
    unsigned flags;
};

struct Strip {
    const double *Min;
    double *Mout;
    const double *Tin;
    double *Tout;
    size_t N;
    int nx, ny, y0, y1, gx;
    unsigned ldoff, stoff;  // byte offsets of the lane's column: loads, stores (kOut on halo lanes)
    bool walls;  // walls at the first and last rows; periodic rows otherwise
    bool interior;
    double sub;
};

__device__ __forceinline__ void set_row(double v, double &c, double &d, double &s)
{
    const double l = from_left(v), r = from_right(v);
    c = v;
    d = r - l;
    s = r + l;
}

// K(T) at a node from the three rows of the field the stage differentiates
// (T^n for the first stage, T~ for the second), centre value t0.
__device__ __forceinline__ double energy_rhs(const Phys &c, double cm, double dm, double sm, double t0,
                                             double d0, double s0, double cp, double dp, double sp,
                                             double ux, double uy, double divu, double inv, double Z)
{
    const double gx = d0 * (1.0 / 3.0) + (dp + dm) * (1.0 / 12.0);
    const double gy = (cp - cm) * (1.0 / 3.0) + (sp - sm) * (1.0 / 12.0);
    const double c4 = 4.0 * t0;
    const double lap = ((s0 + (cp + cm)) - c4) * (2.0 / 3.0) + ((sp + sm) - c4) * (1.0 / 6.0);
    const double adv = -(ux * gx + uy * gy);
    const double cond = c.kappa_over_cv * inv * lap;
    const double work = -t0 * c.R_over_cv * Z * divu;
    return adv + cond + work;
}

// tau = 1 collision: f* = f_eq(rho, u) + F' with Li's forcing, the rest
// population closed by mass conservation (the same expressions as the tile
// kernels' collision).
__device__ __forceinline__ void collide(const Phys &c, double rho, double ux, double uy, double Fx, double Fy,
                                        double X, double fs[9])
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

// Next level's mass of a post-collision set: a population moving into a
// wall layer is counted twice by that wall's reconstruction, one leaving
// through a wall not at all.
__device__ __forceinline__ double next_mass(const double v[9], int gy, int ny, bool walls)
{
    double nm = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])) + v[8];
    if (walls) {
        const double down = (v[4] + v[7]) + v[8], up = (v[2] + v[5]) + v[6];
        nm = gy == 0 ? nm - down : nm;
        nm = gy == 1 ? nm + down : nm;
        nm = gy == ny - 2 ? nm + up : nm;
        nm = gy == ny - 1 ? nm - up : nm;
    }
    return nm;
}

// Diagnostics of a node of level n (mass, max |u|^2, min rho, NaN flag),
// added when the lane owns the node: by selects, or (BRANCH) by a branch,
// which keeps the register demand of the wall segments' steps lower.
template <bool BRANCH>
__device__ __forceinline__ void level_diag(Rings &R, bool own, double rho, double ux, double uy)
{
    const double uu = ux * ux + uy * uy;
    const bool nan = rho != rho || ux != ux || uy != uy;
    if (BRANCH) {
        if (own) {
            R.mass_n += rho;
            R.umax = fmax(R.umax, uu);
            R.rmin = fmin(R.rmin, rho);
            if (nan) R.flags |= kFlagNaN;
        }
    } else {
        R.mass_n += own ? rho : 0.0;
        R.umax = own ? fmax(R.umax, uu) : R.umax;
        R.rmin = own ? fmin(R.rmin, rho) : R.rmin;
        R.flags |= (own && nan) ? kFlagNaN : 0u;
    }
}

// psi and Z(eta) of a node (Eqs. EOS, InteractionPotential), the EOS fixed
// at compile time; the same arithmetic as psi_and_Z.  A row of zeros (beyond
// a wall) gets psi = 0.
template <int EOS>
__device__ __forceinline__ double psi_Z(const Phys &c, double rho, double T, double &Z)
{
    if constexpr (EOS == 1) {
        Z = 0.0;
        return 0.0;
    } else {
        Z = cs_Z(c.b_quarter * rho);
        const double p = rho * (c.R * T * Z - c.a * rho);
        return sqrt_pos_sel(c.two_over_G * (p - rho * (1.0 / 3.0)));
    }
}

// Issue the loads of row r into ring slot S (zeros beyond a wall and past
// the last row the segment reads: every path writes the slot, so that no
// ring value has to outlive its row).
template <bool EDGE, int S>
__device__ __forceinline__ void issue_row(Rings &R, const Strip &A, int r)
{
    // rows past the last one the segment reads, and rows beyond a wall, are
    // read as zeros (an empty range); the row index is uniform
    bool need = r < A.y1 + kHalo;
    int gy = r;
    if (EDGE) {
        if (A.walls) need = need && r >= 0 && r < A.ny;
        else gy = wrap(r, A.ny);
    }
    gy = need ? gy : 0;
    const int bytes = need ? A.nx * 8 : 0;
    const size_t row = (size_t)gy * A.nx;
    R.lr[S] = row_load(A.Min + row, bytes, A.ldoff);
    R.ljx[S] = row_load(A.Min + A.N + row, bytes, A.ldoff);
    R.ljy[S] = row_load(A.Min + 2 * A.N + row, bytes, A.ldoff);
    R.lT[S] = row_load(A.Tin + row, bytes, A.ldoff);
}

// Stages of a march step (a compile-time set: the first and last steps of a
// segment run only the stages whose rows the segment needs).
constexpr int kLoad = 1, kForce = 2, kCollide = 4, kPull = 8, kHeun1 = 16, kHeun2 = 32;
constexpr int kAll = 63;

// One step of the march: loads of row a + kPF, then the stages in PH.  J is
// the ring slot of row a.  A step of an interior segment holds no branch (a
// lane's own nodes select their diagnostics), so that the compiler can
// interleave the independent stages of the step; a segment with a wall row
// branches, uniformly, around the stages that wall rows and the rows of
// zeros beyond them skip.
template <bool EDGE, int EOS, int J, int PH>
__device__ __forceinline__ void march_step(Rings &R, const Strip &A, const Phys &c, int a)
{
    constexpr int S0 = J & 3, S1 = (J + 3) & 3, S2 = (J + 2) & 3, S3 = (J + 1) & 3;  // rows a, a-1, a-2, a-3
    constexpr int S4 = J & 3;                                                       // row a-4
    const bool walls = EDGE && A.walls;
    if (PH & kLoad) issue_row<EDGE, (J + kPF) & 3>(R, A, a + kPF);

    // ---- row a: psi, Z and the stencil rows of psi and T^n ----
    if (PH & kLoad) {
        const double rho = R.lr[S0], T = R.lT[S0];
        double Z;
        const double psi = psi_Z<EOS>(c, rho, T, Z);
        R.rho[S0] = rho;
        R.jx[S0] = R.ljx[S0];
        R.jy[S0] = R.ljy[S0];
        R.Z[S0] = Z;
        set_row(psi, R.pc[S0], R.pd[S0], R.ps[S0]);
        set_row(T, R.tc[S0], R.td[S0], R.ts[S0]);
        const bool own = a >= A.y0 && a < A.y1 && A.interior;
        unsigned fl = (rho > 0.0 ? 0u : kFlagRho) | (psi != psi ? kFlagPsi : 0u);
        if (EOS == 0) fl |= c.b_quarter * rho >= 1.0 ? kFlagEta : 0u;
        R.flags |= own ? fl : 0u;
    }

    if (EDGE) __builtin_amdgcn_sched_barrier(0);  // a wall segment keeps its stages apart
    // ---- row a - 1: force, force-corrected velocity and the collision ----
    const int b = a - 1;
    if (PH & kForce) {
        const double rho = R.rho[S1];
        double Fx = 0.0, Fy = 0.0, X = 0.0, inv = 0.0, ux = 0.0, uy = 0.0;
        if (!walls || (b > 0 && b < A.ny - 1)) {  // wall rows carry no force
            const double sx = R.pd[S1] * (1.0 / 3.0) + (R.pd[S0] + R.pd[S2]) * (1.0 / 12.0);
            const double sy = (R.pc[S0] - R.pc[S2]) * (1.0 / 3.0) + (R.ps[S0] - R.ps[S2]) * (1.0 / 12.0);
            const double mg = -c.G * R.pc[S1];
            Fx = mg * sx;
            Fy = mg * sy + gravity_force(rho, A.sub, c.g);
            X = c.G2 * (sx * sx + sy * sy);
        }
        if (!walls || (b >= 0 && b < A.ny)) {  // rows beyond a wall keep u = 0
            inv = rcp_pos(rho);
            ux = (R.jx[S1] + 0.5 * Fx) * inv;
            uy = (R.jy[S1] + 0.5 * Fy) * inv;
        }
        R.inv[S1] = inv;
        R.ux[S1] = ux;
        R.uy[S1] = uy;
        const double uxl = from_left(ux), uxr = from_right(ux);
        const double uyl = from_left(uy), uyr = from_right(uy);
        R.uxd[S1] = uxr - uxl;
        R.uys[S1] = uyr + uyl;
        const bool own = b >= A.y0 && b < A.y1 && A.interior;
        level_diag<EDGE>(R, own, rho, ux, uy);
        if (PH & kCollide) {
            // tau = 1: the post-collision set of row b is a function of its
            // (rho, u, F, X) alone, so it is formed here; a row of zeros
            // beyond a wall gives a set of zeros (it sends nothing)
            double fs[9];
            collide(c, rho, ux, uy, Fx, Fy, X, fs);
            const double nm = next_mass(fs, b, A.ny, walls);
            R.mass_next += own ? nm : 0.0;
            R.flags |= (own && nm != nm) ? kFlagNaN : 0u;
            // f_i(x) = f*_i(x - c_i): x-components +1 come from the left lane,
            // -1 from the right lane; y-components +1 go to row b + 1, -1 to b - 1
            R.pull[S0][2] = fs[2];
            R.pull[S0][5] = from_left(fs[5]);
            R.pull[S0][6] = from_right(fs[6]);
            R.pull[S1][0] = fs[0];
            R.pull[S1][1] = from_left(fs[1]);
            R.pull[S1][3] = from_right(fs[3]);
            R.pull[S2][4] = fs[4];
            R.pull[S2][7] = from_right(fs[7]);
            R.pull[S2][8] = from_left(fs[8]);
        }
    }

    if (EDGE) __builtin_amdgcn_sched_barrier(0);  // a wall segment keeps its stages apart
    // ---- row a - 2: moments of the pulled set ----
    if (PH & kPull) {
        const int p = a - 2;
        double f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = R.pull[S2][i];
        if (walls && p == 0) {  // Zou-He, bottom wall: unknowns 2, 5, 6
            const double d = f[1] - f[3];
            f[2] = f[4];
            f[5] = f[7] - 0.5 * d;
            f[6] = f[8] + 0.5 * d;
        }
        if (walls && p == A.ny - 1) {  // top wall: unknowns 4, 7, 8
            const double d = f[1] - f[3];
            f[4] = f[2];
            f[7] = f[5] + 0.5 * d;
            f[8] = f[6] - 0.5 * d;
        }
        const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        const double jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
        const double jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
        const size_t row = (size_t)p * A.nx;
        row_store(A.Mout + row, A.nx * 8, A.stoff, rho);
        row_store(A.Mout + A.N + row, A.nx * 8, A.stoff, jx);
        row_store(A.Mout + 2 * A.N + row, A.nx * 8, A.stoff, jy);
    }

    if (EDGE) __builtin_amdgcn_sched_barrier(0);  // a wall segment keeps its stages apart
    // ---- row a - 2: first Heun stage ----
    const int r2 = a - 2;
    if (PH & kHeun1) {
        double k1 = 0.0, dv = 0.0;
        if (!walls || (r2 > 0 && r2 < A.ny - 1)) {
            // rows r2 - 1, r2, r2 + 1 sit in slots S3, S2, S1
            dv = (R.uxd[S2] * (1.0 / 3.0) + (R.uxd[S1] + R.uxd[S3]) * (1.0 / 12.0)) +
                 ((R.uy[S1] - R.uy[S3]) * (1.0 / 3.0) + (R.uys[S1] - R.uys[S3]) * (1.0 / 12.0));
            k1 = energy_rhs(c, R.tc[S3], R.td[S3], R.ts[S3], R.tc[S2], R.td[S2], R.ts[S2], R.tc[S1], R.td[S1],
                            R.ts[S1], R.ux[S2], R.uy[S2], dv, R.inv[S2], R.Z[S2]);
        }
        const double Tt = R.tc[S2] + k1;
        R.k1[S2] = k1;
        R.dv[S2] = dv;
        set_row(Tt, R.ttc[S2], R.ttd[S2], R.tts[S2]);
    }

    if (EDGE) __builtin_amdgcn_sched_barrier(0);  // a wall segment keeps its stages apart
    // ---- row a - 3: second Heun stage and T^{n+1} (always a row of the segment) ----
    if (PH & kHeun2) {
        const int q = a - 3;
        const double T = R.tc[S3];
        double Tn = T;
        if (!walls || (q > 0 && q < A.ny - 1)) {  // wall rows keep their temperature
            // T~ rows q - 1, q, q + 1 sit in slots S4, S3, S2
            const double k2 = energy_rhs(c, R.ttc[S4], R.ttd[S4], R.tts[S4], R.ttc[S3], R.ttd[S3], R.tts[S3],
                                         R.ttc[S2], R.ttd[S2], R.tts[S2], R.ux[S3], R.uy[S3], R.dv[S3],
                                         R.inv[S3], R.Z[S3]);
            Tn = T + 0.5 * (R.k1[S3] + k2);
        }
        row_store(A.Tout + (size_t)q * A.nx, A.nx * 8, A.stoff, Tn);
        R.flags |= (A.interior && Tn != Tn) ? kFlagNaN : 0u;
    }
}

// The march over one segment.
template <bool EDGE, int EOS>
__device__ __forceinline__ void march(const Strip &A, const Phys &c, Partial &part)
{
    // Step a loads row a, takes the force, velocity and collision of row
    // a - 1, the pull and the first Heun stage of row a - 2 and the second
    // Heun stage of row a - 3.  The segment [y0, y1) needs psi on rows
    // y0 - 3 .. y1 + 2, u on y0 - 2 .. y1 + 1, the collision on y0 - 1 ..
    // y1, the first Heun stage on y0 - 1 .. y1 and the rest on its own rows:
    // six entry steps, y1 - y0 - 1 steps with every stage and a last step.
    Rings R;
    R.mass_n = R.mass_next = R.umax = 0.0;
    R.rmin = 1e300;
    R.flags = 0u;
    const int a0 = A.y0 - kHalo;
    issue_row<EDGE, 0>(R, A, a0);
    issue_row<EDGE, 1>(R, A, a0 + 1);
    if constexpr (kPF > 2) issue_row<EDGE, 2>(R, A, a0 + 2);
    march_step<EDGE, EOS, 0, kLoad>(R, A, c, a0);
    march_step<EDGE, EOS, 1, kLoad>(R, A, c, a0 + 1);
    march_step<EDGE, EOS, 2, kLoad | kForce>(R, A, c, a0 + 2);
    march_step<EDGE, EOS, 3, kLoad | kForce | kCollide>(R, A, c, a0 + 3);
    march_step<EDGE, EOS, 0, kLoad | kForce | kCollide | kHeun1>(R, A, c, a0 + 4);
    march_step<EDGE, EOS, 1, kAll & ~kHeun2>(R, A, c, a0 + 5);
    int a = a0 + 6;
    const int last = A.y1 + 1;  // last step with every stage
    for (; a + 3 <= last; a += 4) {
        march_step<EDGE, EOS, 2, kAll>(R, A, c, a);
        march_step<EDGE, EOS, 3, kAll>(R, A, c, a + 1);
        march_step<EDGE, EOS, 0, kAll>(R, A, c, a + 2);
        march_step<EDGE, EOS, 1, kAll>(R, A, c, a + 3);
    }
    constexpr int kLast = kLoad | kForce | kHeun1 | kHeun2;
    switch (last + 1 - a) {
    case 0:
        march_step<EDGE, EOS, 2, kLast>(R, A, c, a);
        break;
    case 1:
        march_step<EDGE, EOS, 2, kAll>(R, A, c, a);
        march_step<EDGE, EOS, 3, kLast>(R, A, c, a + 1);
        break;
    case 2:
        march_step<EDGE, EOS, 2, kAll>(R, A, c, a);
        march_step<EDGE, EOS, 3, kAll>(R, A, c, a + 1);
        march_step<EDGE, EOS, 0, kLast>(R, A, c, a + 2);
        break;
    default:
        march_step<EDGE, EOS, 2, kAll>(R, A, c, a);
        march_step<EDGE, EOS, 3, kAll>(R, A, c, a + 1);
        march_step<EDGE, EOS, 0, kAll>(R, A, c, a + 2);
        march_step<EDGE, EOS, 1, kLast>(R, A, c, a + 3);
        break;
    }
    part.mass_n += R.mass_n;
    part.mass_next += R.mass_next;
    part.umax = fmax(part.umax, R.umax);
    part.rmin = fmin(part.rmin, R.rmin);
    part.flags |= R.flags;
}

template <int EOS>
__global__ __launch_bounds__(kNT, 2) void d2q9_march_mom(const double *__restrict__ Min, double *__restrict__ Mout,
                                                         const double *__restrict__ Tin, double *__restrict__ Tout,
                                                         Phys c, int nx, int ny, int walls, int nstrips, int nseg, int spb,
                                                         double *__restrict__ partials, StepState *__restrict__ st,
                                                         int64_t step)
{
    __shared__ double s_red[4 * kNT / 64];
    __shared__ unsigned s_ured[kNT / 64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // blocks are dealt to the eight XCDs in turn: XCD k takes the k-th band
    // of segments, so that neighbouring strips and segments share its L2
    const int band = blockIdx.x & 7;
    const int i = (int)(blockIdx.x >> 3) * (kNT / 64) + wv;
    const int sib = i / nstrips, strip = i - sib * nstrips;
    const int seg = band * spb + sib;

    Partial part = {0.0, 0.0, 0.0, 1e300, 0u};
    if (sib < spb && seg < nseg) {
        Strip A;
        A.Min = Min;
        A.Mout = Mout;
        A.Tin = Tin;
        A.Tout = Tout;
        A.N = (size_t)nx * ny;
        A.nx = nx;
        A.ny = ny;
        A.walls = walls != 0;
        A.y0 = (int)((int64_t)seg * ny / nseg);
        A.y1 = (int)((int64_t)(seg + 1) * ny / nseg);
        const int x0 = (int)((int64_t)strip * nx / nstrips);
        const int x1 = (int)((int64_t)(strip + 1) * nx / nstrips);
        A.gx = wrap(x0 - kHalo + lane, nx);
        A.interior = lane >= kHalo && lane < kHalo + (x1 - x0);
        A.ldoff = (unsigned)A.gx * 8u;
        A.stoff = A.interior ? A.ldoff : kOut;
        A.sub = gravity_sub(c.form, st->mean[step & 1], c.rho_v);

        // segments whose rows all exist and hold no wall row take the
        // variant without the checks
        if (A.y0 >= kHalo && A.y1 <= ny - kHalo)
            march<false, EOS>(A, c, part);
        else
            march<true, EOS>(A, c, part);
    }
    part = block_reduce<kNT>(part, s_red, s_ured);
    finish_launch<kNT>(part, partials, st, step, (int)((step + 1) & 1), 1.0 / ((double)nx * ny), s_red, s_ured);
}

struct MarchGrid {
    int nstrips, nseg, spb, nblocks;
};

// Strips of at most 58 columns; segments so that the grid holds about two
// wavefronts per SIMD (eight per compute unit), a multiple of 8 once there
// are at least 8, dealt to the XCDs in bands of spb segments.
MarchGrid march_grid(int nx, int ny, int cus)
{
    MarchGrid g;
    g.nstrips = (nx + kStrip - 1) / kStrip;
    const long target = 8L * cus;
    long nseg = target / g.nstrips;
    if (nseg < 1) nseg = 1;
    if (nseg > ny) nseg = ny;
    if (nseg >= 8) nseg -= nseg % 8;
    g.nseg = (int)nseg;
    g.spb = (g.nseg + 7) / 8;
    g.nblocks = 8 * ((g.spb * g.nstrips + kNT / 64 - 1) / (kNT / 64));
    return g;
}

}  // namespace

int d2q9_march_blocks(int nx, int ny, int cus) { return march_grid(nx, ny, cus).nblocks; }

hipError_t d2q9_march_launch(const LatticeLaunch &L)
{
    const MarchGrid g = march_grid(L.nx, L.ny, L.resident);
    auto kern = L.phys.eos == 1 ? d2q9_march_mom<1> : d2q9_march_mom<0>;
    hipLaunchKernelGGL(kern, dim3(g.nblocks), dim3(kNT), 0, L.stream, (const double *)L.fin,
                       (double *)L.fout, L.Tin, L.Tout, L.phys, L.nx, L.ny, L.walls ? 1 : 0, g.nstrips, g.nseg,
                       g.spb, L.partials, L.st, L.step);
    return hipGetLastError();
}

}  // namespace tplbm
