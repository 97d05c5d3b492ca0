// D3Q19 update (every relaxation time 1) as two z-marching kernels: L (the
// population state: FP32 deviations or FP64 populations) or LM (the FP64
// moment state, described above its kernel), then E.
//
// A block owns a 32 x 16 tile of (x, y) columns and a range of z planes (a
// segment), and walks the planes upwards keeping one thread per column.  The
// planes of the fields a stencil needs are staged in LDS, so each field is
// read from memory once per node; the halo of a tile is the ring of columns
// around it.
//
//   L (halo 1): pull f_i(x) = f*_i(x - c_i) of the previous level with the
//     wet-node reconstruction on wall planes, rho and j (Eqs. Density,
//     Momentum), psi (Eqs. EOS, InteractionPotential) -> a ring of four psi
//     planes in LDS.  One plane behind: the Shan-Chen force (Eq.
//     ShanChenForce, zero on wall planes) and gravity (Eqs. Gravity_*), u =
//     (j + F/2)/rho, and the tau = 1 collision (f_eq plus half of Guo's term
//     plus the isotropic sigma term), stored as the next level's f*; u and
//     rho go to U for E (LM: u only); the diagnostics of the level (mass with wall
//     multiplicities for <rho>, max |u|, min rho, flags) are reduced as in
//     the other lattice kernels.
//   E (halo 2): the energy equation (Eq. Energy_Equation) advanced by
//     Heun's method with rho and u of the level frozen: T^n and u planes in
//     LDS; one plane behind, div u and k1 = K(T^n) on the tile and its halo
//     ring, T~ = T^n + k1 -> LDS; two more planes behind, k2 = K(T~) and
//     T^{n+1} = T^n + (k1 + k2)/2 on the tile.  Wall planes keep T.  One
//     barrier per plane: the second stage reads only T~ planes written
//     before it.
//
// The divergence of u is accumulated plane by plane: the contribution of a
// plane to the divergence at its own plane and at the planes above and below
// depends only on that plane's values, so u needs a single plane in LDS.
//
// Threads and columns: in L thread t owns interior column t (x = t % 32, y =
// t / 32 of the tile) and threads 0..99 take the ring of columns at distance 1
// as a second column; a block of 512 threads (8 waves, one block per compute
// unit) leaves each thread up to 256 registers for the loads of the next
// plane in flight.  In E every thread has one column: the tile's 512, then
// the 100 of the ring at distance 1, then the 108 at distance 2.  Column
// coordinates wrap in x and y (periodic), so a tile that extends past the
// lattice edge reads the periodic images; only columns inside the lattice
// store results.
#include <hip/hip_runtime.h>

#include "d3q19_common.hpp"
#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {

using namespace d3;

// A tile of TX x TY columns and the rings of Ring1 and Ring2 columns at
// distance 1 and 2 around it.  Region<H> is the tile with a halo of H
// columns, kept in LDS with an odd row stride RX (in doubles), so that a run
// of columns down the region's sides (the ring columns) falls into distinct
// banks.
template <int TX_, int TY_>
struct Tile {
    static constexpr int TX = TX_, TY = TY_, Threads = TX * TY;
    static constexpr int Ring1 = 2 * (TX + 2) + 2 * TY, Ring2 = 2 * (TX + 4) + 2 * (TY + 2);
    template <int H>
    struct Region {
        static constexpr int W = TX + 2 * H, RY = TY + 2 * H, RX = W + 1, N = RX * RY;
    };
};
// L: 512 threads (8 waves, one block per compute unit), leaving each thread up
// to 256 registers for the pulled populations of the next plane in flight.
// E: 720 threads (12 waves, one block per compute unit), one column each.
using TileL = Tile<32, 16>;
using TileE = Tile<32, 16>;
static_assert(TileL::Ring1 <= TileL::Threads, "L's ring at distance 1 is taken as a second column");

// Region coordinates of column k of the ring at distance r from the tile,
// inside a region of halo H >= r: bottom row, top row, left and right sides.
template <class T>
__device__ __forceinline__ void ring_column(int r, int H, int k, int &rx, int &ry)
{
    const int w = T::TX + 2 * r, h = T::TY + 2 * r, off = H - r;
    if (k < w) {
        rx = k;
        ry = 0;
    } else if (k < 2 * w) {
        rx = k - w;
        ry = h - 1;
    } else if (k < 2 * w + (h - 2)) {
        rx = 0;
        ry = 1 + (k - 2 * w);
    } else {
        rx = w - 1;
        ry = 1 + (k - 2 * w - (h - 2));
    }
    rx += off;
    ry += off;
}

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Population-plane accesses through buffer resources: the base address of a
// z layer of a population plane is uniform (scalar registers) and a lane's
// column offset within the layer goes in the vector offset, so an access
// costs no vector address arithmetic.  Offsets are in bytes within one layer.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dword access (gfx9 family)

// one z layer (nx ny nodes) of a population plane; its base moves with the
// layer, so the resources are formed per layer rather than held across the
// march
template <class S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t layer_rsrc(const S *base, unsigned plane)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(plane * (unsigned)sizeof(S)), kRsrcWord3);
}
// the same with an empty range when `none` (a layer beyond a wall): its
// loads return zero without a memory access
template <class S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t layer_rsrc(const S *base, unsigned plane, bool none)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, none ? 0 : (int)(plane * (unsigned)sizeof(S)),
                                             kRsrcWord3);
}
// added to a lane's byte offset, it puts the access out of every layer's
// range (loads return zero, stores are dropped): lanes without a second
// column
constexpr unsigned kOut = 0x80000000u;
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// Stores are non-temporal (cache-policy bit 1): nothing a step writes is read
// again before it has left the L2, and streaming the writes past it measured
// 5% faster for the whole step; loads keep the default policy, since the
// halo columns of neighbouring tiles are re-read from the L2.
constexpr int kStoreNT = 2;
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, kStoreNT);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, kStoreNT);
}
// store a population value (as an FP32 deviation from wr, or FP64) and
// return it as stored
__device__ __forceinline__ double pop_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v, double wr,
                                         float)
{
    const float d = (float)(v - wr);
    buf_st(r, voff, soff, d);
    return wr + (double)d;
}
__device__ __forceinline__ double pop_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v, double,
                                         double)
{
    buf_st(r, voff, soff, v);
    return v;
}

// Block -> tile and z segment.  Blocks are dealt to the eight XCDs in turn;
// XCD k takes the k-th contiguous eighth of the (segment-major) block list,
// so the tiles one XCD runs together are neighbours in x and y of the same
// segment and share their halo columns in its L2.
struct MarchG3 {
    int ntx, nty, nseg, nblocks;
};

struct Seg3 {
    int x0, y0, z0, z1;
};

template <class T>
__device__ __forceinline__ Seg3 block_segment(const MarchG3 &M, int nz)
{
    const int nb = M.nblocks;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tiles = M.ntx * M.nty;
    const int seg = b / tiles, tl = b - seg * tiles;
    Seg3 s;
    s.x0 = (tl % M.ntx) * T::TX;
    s.y0 = (tl / M.ntx) * T::TY;
    s.z0 = (int)((int64_t)seg * nz / M.nseg);
    s.z1 = (int)((int64_t)(seg + 1) * nz / M.nseg);
    return s;
}

// Plane index of z for loads: wrapped (periodic) or clamped to the wall
// planes (walls).  `beyond` tells a plane outside a walled lattice.
template <bool WALLS>
__device__ __forceinline__ int plane_of(int z, int nz, bool &beyond)
{
    if (WALLS) {
        beyond = z < 0 || z >= nz;
        return z < 0 ? 0 : (z >= nz ? nz - 1 : z);
    }
    beyond = false;
    return wrap_mod(z, nz);
}

// Column of a tile's region: its node offsets within a plane for dx, dy in
// {-1, 0, 1} (periodic x, y), and whether it is a lattice node this block
// owns (interior columns inside the lattice).
struct Col {
    unsigned xo[3];   // x + dx, wrapped
    unsigned yo[3];   // (y + dy, wrapped) * nx
    unsigned n0;      // yo[1] + xo[1]
    unsigned oob;     // 0, or kOut for a lane that has no such column
    int r;            // region index
};

__device__ __forceinline__ Col make_col(const Grid3 &G, int x0, int y0, int rx, int ry, int H, int RX,
                                        bool exists = true)
{
    Col c;
    c.oob = exists ? 0u : kOut;
    const int gx = x0 + rx - H, gy = y0 + ry - H;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c.xo[d] = (unsigned)wrap_mod(gx + d - 1, G.nx);
        c.yo[d] = (unsigned)wrap_mod(gy + d - 1, G.ny) * (unsigned)G.nx;
    }
    c.n0 = c.yo[1] + c.xo[1];
    c.r = ry * RX + rx;
    return c;
}

// Shan-Chen sum s = sum_i w(|c_i|^2) psi(x + c_i) c_i (w(1) = 1/6, w(2) =
// 1/12) from three LDS planes of psi (below, own, above) at region index r,
// the neighbours grouped as in grad_lap_planes
template <int RX>
__device__ __forceinline__ void sc_sum_planes(const double *__restrict__ pm, const double *__restrict__ p0,
                                              const double *__restrict__ pp, int r, double &sx, double &sy,
                                              double &sz)
{
    const double ea = p0[r + 1 + RX], eb = p0[r + 1 - RX], ec = p0[r - 1 + RX], ed = p0[r - 1 - RX];
    const double bxp = pm[r + 1], bxm = pm[r - 1], byp = pm[r + RX], bym = pm[r - RX];
    const double axp = pp[r + 1], axm = pp[r - 1], ayp = pp[r + RX], aym = pp[r - RX];
    const double ex = ((ea + eb) - (ec + ed)) + ((bxp - bxm) + (axp - axm));
    const double ey = ((ea - eb) + (ec - ed)) + ((byp - bym) + (ayp - aym));
    const double ez = ((axp + axm) + (ayp + aym)) - ((bxp + bxm) + (byp + bym));
    sx = (1.0 / 6.0) * (p0[r + 1] - p0[r - 1]) + (1.0 / 12.0) * ex;
    sy = (1.0 / 6.0) * (p0[r + RX] - p0[r - RX]) + (1.0 / 12.0) * ey;
    sz = (1.0 / 6.0) * (pp[r] - pm[r]) + (1.0 / 12.0) * ez;
}

// ---- L: pull, psi, force, u, collision -------------------------------------

// Loads of one column at one plane: the nineteen pulled values f*_i(x - c_i)
// as stored, and T.  Issued one plane ahead of their use.
template <class S>
struct PullLoads {
    S f[19];
    double T;
};

template <class S, bool WALLS>
__device__ __forceinline__ void pull_issue(PullLoads<S> &P, const S *__restrict__ fin,
                                           const double *__restrict__ Tin, const Grid3 &G, const Col &c, int a)
{
    // a plane beyond a wall reads zeros (an empty range): no branch, so the
    // loads stay in flight across the step that issues them
    bool beyond;
    const int za = plane_of<WALLS>(a, G.nz, beyond);
    const unsigned plane = (unsigned)G.nx * (unsigned)G.ny;
    unsigned zoff[3];  // zoff[1 - c_z]: the plane a - c_z a population comes from
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bool bb;
        zoff[d] = (unsigned)plane_of<WALLS>(za + d - 1, G.nz, bb) * plane;
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const V3 v = vel(i);
        P.f[i] = buf_ld(layer_rsrc(fin + (size_t)i * G.N + zoff[1 - v.z], plane, beyond),
                        (c.yo[1 - v.y] + c.xo[1 - v.x]) * (unsigned)sizeof(S) + c.oob, 0u, S());
    }
    P.T = buf_ld(layer_rsrc(Tin + zoff[1], plane, beyond), c.n0 * 8u + c.oob, 0u, 0.0);
}

// rho, j (wall reconstruction on wall planes) and psi of a pulled column
template <class S, bool WALLS>
__device__ __forceinline__ double pull_finish(const PullLoads<S> &P, const Phys &c, const Grid3 &G, int a,
                                              const double *__restrict__ rref, double &rho, double &jx, double &jy,
                                              double &jz)
{
    bool beyond;
    const int za = plane_of<WALLS>(a, G.nz, beyond);
    double rz[3] = {0.0, 0.0, 0.0};
    if (sizeof(S) == 4) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            bool bb;
            rz[d] = rref[plane_of<WALLS>(za + d - 1, G.nz, bb)];
        }
    }
    double f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = Pop<S>::val(P.f[i], wgt(i) * rz[1 - vel(i).z]);
    // the zero-velocity wet-node reconstruction of the populations from
    // beyond a wall (with transverse momentum corrections), written out here:
    // passed to a function by reference, the array would be kept in private
    // memory, whose accesses share the wait counter of the loads in flight
    if (WALLS && (za == 0 || za == G.nz - 1)) {
        const int s = za == 0 ? 1 : -1;
        double Nx = 0.0, Ny = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const V3 v = vel(i);
            if (v.z == 0) {
                if (v.x) Nx += 0.5 * v.x * f[i];
                if (v.y) Ny += 0.5 * v.y * f[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const V3 v = vel(i);
            if (v.z == s) {
                double r = f[opp(i)];
                if (v.x) r -= (double)v.x * Nx;
                if (v.y) r -= (double)v.y * Ny;
                f[i] = r;
            }
        }
    }
    rho = jx = jy = jz = 0.0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const V3 v = vel(i);
        rho += f[i];
        if (v.x) jx += v.x * f[i];
        if (v.y) jy += v.y * f[i];
        if (v.z) jz += v.z * f[i];
    }
    double Z;
    const double psi = psi_and_Z(c, rho, P.T, Z);
    // a plane beyond a wall holds nothing (its values feed no stencil that
    // is evaluated)
    rho = beyond ? 0.0 : rho;
    jx = beyond ? 0.0 : jx;
    jy = beyond ? 0.0 : jy;
    jz = beyond ? 0.0 : jz;
    return beyond ? 0.0 : psi;
}

template <class S, bool WALLS>
__global__ __launch_bounds__(TileL::Threads) void d3q19_march_l(const S *__restrict__ fin, S *__restrict__ fout,
                                                          const double *__restrict__ Tin, double *__restrict__ U,
                                                          Phys c, Grid3 G, MarchG3 M, double *__restrict__ partials,
                                                          StepState *__restrict__ st, int64_t step,
                                                          const double *__restrict__ rref)
{
    using T = TileL;
    using R = T::Region<1>;
    __shared__ double s_psi[4][R::N];
    __shared__ double s_red[4 * T::Threads / 64];
    __shared__ unsigned s_ured[T::Threads / 64];
    const int t = threadIdx.x;
    const unsigned N = G.N;
    const Seg3 sg = block_segment<T>(M, G.nz);
    const int tx = t % T::TX, ty = t / T::TX;
    const Col own = make_col(G, sg.x0, sg.y0, tx + 1, ty + 1, 1, R::RX);
    const bool mine = sg.x0 + tx < G.nx && sg.y0 + ty < G.ny;  // a lattice node of this tile
    const bool has2 = t < T::Ring1;
    int rx2 = 0, ry2 = 0;
    if (has2) ring_column<T>(1, 1, t, rx2, ry2);
    const Col two = make_col(G, sg.x0, sg.y0, rx2, ry2, 1, R::RX, has2);
    const double sub = gravity_sub(c.form, st->mean[step & 1], c.rho_v);
    const unsigned plane = (unsigned)G.nx * (unsigned)G.ny;

    Partial part = {0.0, 0.0, 0.0, 1e300, 0u};
    double rho_b = 0.0, jx_b = 0.0, jy_b = 0.0, jz_b = 0.0;  // plane a - 1 of the own column
    // planes z0 - 1 .. z1 are pulled; the force, velocity and collision of
    // plane a - 1 follow the pull of plane a
    PullLoads<S> pre;
    pull_issue<S, WALLS>(pre, fin, Tin, G, own, sg.z0 - 1);
    for (int a = sg.z0 - 1; a <= sg.z1; ++a) {
        // the ring column's loads are issued first and waited for last (on
        // lanes without one they are out of range); the own column's loads
        // of plane a + 1 are issued before the plane's first use of memory
        // results
        PullLoads<S> rg;
        pull_issue<S, WALLS>(rg, fin, Tin, G, two, a);
        double rho, jx, jy, jz;
        const double psi = pull_finish<S, WALLS>(pre, c, G, a, rref, rho, jx, jy, jz);
        pull_issue<S, WALLS>(pre, fin, Tin, G, own, a + 1);
        s_psi[a & 3][own.r] = psi;
        if (has2) {
            double r2, x2, y2, z2;
            s_psi[a & 3][two.r] = pull_finish<S, WALLS>(rg, c, G, a, rref, r2, x2, y2, z2);
        }
        __syncthreads();

        // plane b = a - 1: force, velocity, collision.  Every lane computes;
        // stores of a plane outside the segment (an empty range) and of
        // lanes outside the lattice (an out-of-range offset) are dropped, so
        // no memory access sits in a branch.
        const int b = a - 1;
        const bool live = b >= sg.z0;  // uniform
        const bool keep = live && mine;
        {
            const int bz = live ? b : sg.z0;
            const bool wall = WALLS && (b == 0 || b == G.nz - 1);
            double Fx = 0.0, Fy = 0.0, Fz = 0.0, Xs2 = 0.0;
            const double psi0 = s_psi[b & 3][own.r];
            if (!wall) {
                double sx, sy, sz;
                sc_sum_planes<R::RX>(s_psi[(b - 1) & 3], s_psi[b & 3], s_psi[(b + 1) & 3], own.r, sx, sy, sz);
                const double mg = -c.G * psi0;
                Fx = mg * sx;
                Fy = mg * sy;
                Fz = mg * sz + gravity_force(rho_b, sub, c.g);
                Xs2 = c.sigma * c.G2 * (sx * sx + sy * sy + sz * sz);  // sigma |F_int|^2 / psi^2
            }
            const double inv = rcp_pos(rho_b);
            const double ux = (jx_b + 0.5 * Fx) * inv, uy = (jy_b + 0.5 * Fy) * inv, uz = (jz_b + 0.5 * Fz) * inv;
            const size_t zb = (size_t)bz * plane;
            const unsigned vo = own.n0 * 8u + (mine ? 0u : kOut);
            buf_st(layer_rsrc(U + zb, plane, !live), vo, 0u, ux);
            buf_st(layer_rsrc(U + N + zb, plane, !live), vo, 0u, uy);
            buf_st(layer_rsrc(U + 2 * (size_t)N + zb, plane, !live), vo, 0u, uz);
            buf_st(layer_rsrc(U + 3 * (size_t)N + zb, plane, !live), vo, 0u, rho_b);
            const double uu = ux * ux + uy * uy + uz * uz;
            const double uF = ux * Fx + uy * Fy + uz * Fz;
            // post-collision populations (f_eq + half of Guo's term + the
            // sigma term) of each velocity pair c, -c from their even and odd
            // parts, stored as they are formed; the rest population closes
            // the mass
            const double rr = sizeof(S) == 4 ? rref[bz] : 0.0;  // this plane's reference (FP32)
            const unsigned pvo = own.n0 * (unsigned)sizeof(S) + (mine ? 0u : kOut);
            const double even0 = rho_b * (1.0 - 1.5 * uu) - 1.5 * uF, sig2 = 0.75 * Xs2;
            double rest = 0.0, nm = 0.0, down = 0.0, up = 0.0;
#pragma unroll
            for (int i = 1; i < 19; i += 2) {
                const V3 v = vel(i);
                const double w = wgt(i);
                const double cu = cdot(v, ux, uy, uz), cF = cdot(v, Fx, Fy, Fz);
                const double E = w * (even0 + 4.5 * cu * (rho_b * cu + cF) + (i < 7 ? 0.0 : sig2));
                const double O = w * (3.0 * rho_b * cu + 1.5 * cF);
                const double fp = E + O, fm = E - O;
                rest += fp + fm;
                const double sp =
                    pop_st(layer_rsrc(fout + (size_t)i * N + zb, plane, !live), pvo, 0u, fp, w * rr, S());
                const double sm =
                    pop_st(layer_rsrc(fout + (size_t)(i + 1) * N + zb, plane, !live), pvo, 0u, fm, w * rr, S());
                nm += sp + sm;
                // i + 1 is the opposite velocity of i
                if (v.z < 0) down += sp;
                if (v.z > 0) up += sp;
                if (v.z > 0) down += sm;
                if (v.z < 0) up += sm;
            }
            nm += pop_st(layer_rsrc(fout + zb, plane, !live), pvo, 0u, rho_b - rest, wgt(0) * rr, S());
            if (WALLS) {
                nm = b == 0 ? nm - down : nm;
                nm = b == 1 ? nm + down : nm;
                nm = b == G.nz - 2 ? nm + up : nm;
                nm = b == G.nz - 1 ? nm - up : nm;
            }
            unsigned fl = 0u;
            if (!(rho_b > 0.0)) fl |= kFlagRho;
            if (c.eos == 0 && c.b_quarter * rho_b >= 1.0) fl |= kFlagEta;
            if (psi0 != psi0) fl |= kFlagPsi;
            if (rho_b != rho_b || uu != uu || nm != nm) fl |= kFlagNaN;
            part.mass_n += keep ? rho_b : 0.0;
            part.mass_next += keep ? nm : 0.0;
            part.umax = keep ? fmax(part.umax, uu) : part.umax;
            part.rmin = keep ? fmin(part.rmin, rho_b) : part.rmin;
            part.flags |= keep ? fl : 0u;
        }
        rho_b = rho;
        jx_b = jx;
        jy_b = jy;
        jz_b = jz;
    }
    part = block_reduce<T::Threads>(part, s_red, s_ured);
    finish_launch<T::Threads>(part, partials, st, step, (int)((step + 1) & 1), 1.0 / (double)N, s_red, s_ured);
}

// ---- E: the energy equation --------------------------------------------------

// Per-plane contributions of u to div u = 3 sum_i w_i c_i . u(x + c_i):
// cen to the plane itself (in-plane neighbours), side to the planes above and
// below (their in-plane x, y offsets), zc with + to the plane below and - to
// the plane above (the z components).
struct DivPart {
    double cen, side, zc;
};

template <int RX>
__device__ __forceinline__ DivPart div_part(const double *__restrict__ ux, const double *__restrict__ uy,
                                            const double *__restrict__ uz, int r)
{
    constexpr double w1 = 1.0 / 18.0, w2 = 1.0 / 36.0;
    const double dx = ux[r + 1] - ux[r - 1];
    const double dxy = (ux[r + 1 + RX] - ux[r - 1 + RX]) + (ux[r + 1 - RX] - ux[r - 1 - RX]);
    const double dy = uy[r + RX] - uy[r - RX];
    const double dyx = (uy[r + RX + 1] - uy[r - RX + 1]) + (uy[r + RX - 1] - uy[r - RX - 1]);
    const double s4 = (uz[r + 1] + uz[r - 1]) + (uz[r + RX] + uz[r - RX]);
    DivPart p;
    p.cen = (w1 * dx + w2 * dxy) + (w1 * dy + w2 * dyx);
    p.side = w2 * (dx + dy);
    p.zc = w1 * uz[r] + w2 * s4;
    return p;
}

// Isotropic gradient and Laplacian of a field from three LDS planes (below,
// own, above) at region index r: grad = 3 sum w c phi, lap = 6 sum w (phi_i -
// phi_0).  The eighteen neighbours are grouped so that the components share
// their partial sums: the four in-plane edges through (a + b) -+ (c + d) and
// (a - b) + (c - d), the four edges above and below through their x and y
// differences and their sum, the six axis neighbours through differences
// and one sum (6 w_1 + 12 w_2 = 2/3 multiplies phi_0).
template <int RX>
__device__ __forceinline__ void grad_lap_planes(const double *__restrict__ pm, const double *__restrict__ p0,
                                                const double *__restrict__ pp, int r, double &gx, double &gy,
                                                double &gz, double &lap)
{
    constexpr double w1 = 1.0 / 18.0, w2 = 1.0 / 36.0;
    const double c0 = p0[r];
    // in-plane edges (+1, +1), (+1, -1), (-1, +1), (-1, -1)
    const double ea = p0[r + 1 + RX], eb = p0[r + 1 - RX], ec = p0[r - 1 + RX], ed = p0[r - 1 - RX];
    const double s1 = ea + eb, s2 = ec + ed;
    const double exy_x = s1 - s2, exy_y = (ea - eb) + (ec - ed), exy_s = s1 + s2;
    // edges below and above: (+-1, 0, -+1) and (0, +-1, -+1)
    const double bxp = pm[r + 1], bxm = pm[r - 1], byp = pm[r + RX], bym = pm[r - RX];
    const double axp = pp[r + 1], axm = pp[r - 1], ayp = pp[r + RX], aym = pp[r - RX];
    const double bs = (bxp + bxm) + (byp + bym), as = (axp + axm) + (ayp + aym);
    // axis neighbours
    const double xp = p0[r + 1], xm = p0[r - 1], yp = p0[r + RX], ym = p0[r - RX], zp = pp[r], zm = pm[r];
    const double ax_s = ((xp + xm) + (yp + ym)) + (zp + zm);
    gx = (3.0 * w1) * (xp - xm) + (3.0 * w2) * (exy_x + ((bxp - bxm) + (axp - axm)));
    gy = (3.0 * w1) * (yp - ym) + (3.0 * w2) * (exy_y + ((byp - bym) + (ayp - aym)));
    gz = (3.0 * w1) * (zp - zm) + (3.0 * w2) * (as - bs);
    lap = (6.0 * w1) * ax_s + (6.0 * w2) * (exy_s + (bs + as)) - 4.0 * c0;
}

// div u of a column accumulated over the planes: when the contributions of
// plane a arrive, div(a - 1) = pend + side(a) + zc(a) is complete and pend
// becomes cen(a) + side(a - 1) - zc(a - 1), the part of div(a) known so far.
struct DivAcc {
    double pend, side, zc;
    __device__ __forceinline__ double push(const DivPart &p)
    {
        const double done = pend + p.side + p.zc;
        pend = p.cen + side - zc;
        side = p.side;
        zc = p.zc;
        return 3.0 * done;
    }
};

// The energy-equation coefficients of a node with rho and u frozen: K(phi) =
// -u . grad phi + a1 lap phi - phi a2 with a1 = kappa/(rho c_v) and a2 = (R/c_v)
// Z(eta) div u (Z = 0 for the ideal gas).
struct ECoef {
    double ux, uy, uz, a1, a2;
};

__device__ __forceinline__ ECoef energy_coef(const Phys &c, double ux, double uy, double uz, double rho, double divu)
{
    const double Z = c.eos == 0 ? cs_Z(c.b_quarter * rho) : 0.0;
    return ECoef{ux, uy, uz, c.kappa_over_cv * rcp_pos(rho), c.R_over_cv * Z * divu};
}

__device__ __forceinline__ double energy_k(const ECoef &k, double phi0, double gx, double gy, double gz, double lap)
{
    return -(k.ux * gx + k.uy * gy + k.uz * gz) + k.a1 * lap - phi0 * k.a2;
}

// E runs one column per thread: the tile's columns first (threads 0 .. TX TY
// - 1), then the ring at distance 1, then the ring at distance 2 (loads
// only), so that the waves of the second stage hold tile columns only and
// no thread carries a second column.  One block (12 waves) per compute unit.
constexpr int kEThreads = TileE::Threads + TileE::Ring1 + TileE::Ring2;
constexpr int kEBlocksPerCU = 1;

template <bool WALLS>
__global__ __launch_bounds__(kEThreads) void d3q19_march_e(const double *__restrict__ Tin,
                                                                        double *__restrict__ Tout,
                                                                        const double *__restrict__ U,
                                                                        const double *__restrict__ Rho, Phys c,
                                                                        Grid3 G, MarchG3 M)
{
    using T = TileE;
    using R2 = T::Region<2>;
    using R1 = T::Region<1>;
    // rings of planes indexed by z & 3 (z & 1 for u): the step of plane a
    // writes T and u of plane a, then after its one barrier reads T of a - 2
    // .. a, u of a, and T~ of a - 4 .. a - 2, and writes T~ of a - 1; every
    // slot a step writes was last read before a barrier that lies between
    // that read and the write
    __shared__ double s_T[4][R2::N];
    __shared__ double s_u[2][3][R2::N];
    __shared__ double s_Tt[4][R1::N];
    const int t = threadIdx.x;
    const unsigned N = G.N;
    const Seg3 sg = block_segment<T>(M, G.nz);
    const bool tile = t < T::Threads, ring1 = !tile && t < T::Threads + T::Ring1;
    const bool first = tile || ring1;  // a column of the first stage
    int rx, ry;
    if (tile) {
        rx = t % T::TX + 2;
        ry = t / T::TX + 2;
    } else if (ring1) {
        ring_column<T>(1, 2, t - T::Threads, rx, ry);
    } else {
        ring_column<T>(2, 2, t - T::Threads - T::Ring1, rx, ry);
    }
    const Col col = make_col(G, sg.x0, sg.y0, rx, ry, 2, R2::RX);
    const int r1 = (ry - 1) * R1::RX + (rx - 1);  // index in the region of halo 1 (first-stage columns)
    const bool mine = tile && sg.x0 + rx - 2 < G.nx && sg.y0 + ry - 2 < G.ny;
    const unsigned plane = (unsigned)G.nx * (unsigned)G.ny;
    const unsigned vo = col.n0 * 8u;
    const unsigned vrho = first ? vo : kOut;   // rho is read where the first stage runs
    const unsigned vst = mine ? vo : kOut;     // T^{n+1} is stored by the tile's lattice columns

    DivAcc dv = {0.0, 0.0, 0.0};
    double Tp = 0.0, uxp = 0.0, uyp = 0.0, uzp = 0.0, rhop = 0.0;  // the column's values of plane a - 1
    // second-stage inputs of planes a - 2 (h1) and a - 3 (h2): T^n, k1 and
    // the coefficients, from the first stage of those planes
    double hT1 = 0.0, hk1 = 0.0, hT2 = 0.0, hk2 = 0.0;
    ECoef hc1 = {0.0, 0.0, 0.0, 0.0, 0.0}, hc2 = {0.0, 0.0, 0.0, 0.0, 0.0};
    double pendT = 0.0;  // T^{n+1} of plane pendq (none: pendq < z0), stored in the next step
    int pendq = -1;
    // planes z0 - 2 .. z1 + 1 are read, one plane ahead of their use; a read
    // beyond them is an empty range
    auto load = [&](int z, double &vT, double &vx, double &vy, double &vz, double &vr) __attribute__((always_inline)) {
        bool beyond;
        const size_t zo = (size_t)plane_of<WALLS>(z, G.nz, beyond) * plane;
        beyond = beyond || z > sg.z1 + 1;
        vT = buf_ld(layer_rsrc(Tin + zo, plane, beyond), vo, 0u, 0.0);
        vx = buf_ld(layer_rsrc(U + zo, plane, beyond), vo, 0u, 0.0);
        vy = buf_ld(layer_rsrc(U + N + zo, plane, beyond), vo, 0u, 0.0);
        vz = buf_ld(layer_rsrc(U + 2 * (size_t)N + zo, plane, beyond), vo, 0u, 0.0);
        vr = buf_ld(layer_rsrc(Rho + zo, plane, beyond), vrho, 0u, 0.0);
    };
    double nT, nx, ny, nzv, nr;
    load(sg.z0 - 2, nT, nx, ny, nzv, nr);
    for (int a = sg.z0 - 2; a <= sg.z1 + 2; ++a) {
        s_T[a & 3][col.r] = nT;
        s_u[a & 1][0][col.r] = nx;
        s_u[a & 1][1][col.r] = ny;
        s_u[a & 1][2][col.r] = nzv;
        const double Ta = nT, uxa = nx, uya = ny, uza = nzv, rhoa = nr;
        // the previous step's T^{n+1}, stored ahead of this step's loads so
        // that waiting for those never waits for the store; a plane outside
        // the segment is an empty range
        buf_st(layer_rsrc(Tout + (size_t)(pendq >= sg.z0 ? pendq : sg.z0) * plane, plane, pendq < sg.z0), vst, 0u,
               pendT);
        load(a + 1, nT, nx, ny, nzv, nr);
        __syncthreads();

        // the contributions of plane a complete div u of plane b = a - 1;
        // then the first stage there: k1 = K(T^n), T~ = T^n + k1 (wall
        // planes and the planes beyond them keep T)
        const int b = a - 1;
        double k1b = 0.0;
        ECoef cb = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (first) {
            const double divb = dv.push(div_part<R2::RX>(s_u[a & 1][0], s_u[a & 1][1], s_u[a & 1][2], col.r));
            if (b >= sg.z0 - 1 && b <= sg.z1) {  // uniform
                double Tt = Tp;
                if (!(WALLS && (b <= 0 || b >= G.nz - 1))) {
                    cb = energy_coef(c, uxp, uyp, uzp, rhop, divb);
                    double gx, gy, gz, lap;
                    grad_lap_planes<R2::RX>(s_T[(b - 1) & 3], s_T[b & 3], s_T[a & 3], col.r, gx, gy, gz, lap);
                    k1b = energy_k(cb, Tp, gx, gy, gz, lap);
                    Tt = Tp + k1b;
                }
                s_Tt[b & 3][r1] = Tt;
            }
        }

        // second stage of plane q = a - 3 on the tile: k2 = K(T~), T^{n+1} =
        // T^n + (k1 + k2)/2 (wall planes keep T).  T~ of q + 1 was written
        // in the previous step, before this step's barrier.
        const int q = a - 3;
        if (tile) {
            double gx, gy, gz, lap;
            grad_lap_planes<R1::RX>(s_Tt[(q - 1) & 3], s_Tt[q & 3], s_Tt[(q + 1) & 3], r1, gx, gy, gz, lap);
            const double k2 = energy_k(hc2, s_Tt[q & 3][r1], gx, gy, gz, lap);
            const bool wq = WALLS && (q == 0 || q == G.nz - 1);
            pendT = wq ? hT2 : hT2 + 0.5 * (hk2 + k2);
            pendq = (q >= sg.z0 && q < sg.z1) ? q : -1;
        }
        hT2 = hT1;
        hk2 = hk1;
        hc2 = hc1;
        hT1 = Tp;
        hk1 = k1b;
        hc1 = cb;
        Tp = Ta;
        uxp = uxa;
        uyp = uya;
        uzp = uza;
        rhop = rhoa;
    }
    buf_st(layer_rsrc(Tout + (size_t)(pendq >= sg.z0 ? pendq : sg.z0) * plane, plane, pendq < sg.z0), vst, 0u,
           pendT);
}

// ---- LM: the moment-state step (FP64, every tau = 1) --------------------------

// With every relaxation time 1 the post-collision set of a node is a closed
// function of its (rho, u, F, X), so the state carried between steps can be
// (rho, j) and T instead of the nineteen populations.  LM takes the LBM part
// of a step on that state and hands u to E through U (E reads rho from the
// state itself, which L's populations cannot give it).  One
// column per thread (the tile, the ring at distance 1, the ring at distance
// 2); per plane a:
//   psi of plane a on every column (rho and T read one plane ahead) -> a ring
//     of four psi planes;
//   two planes behind, on the tile and the first ring: the Shan-Chen force
//     and gravity of plane b = a - 2 (zero on wall planes), u = (j + F/2)/rho
//     and X = sigma |F_int|^2 / psi^2 -> the velocity-independent terms of
//     the node's post-collision populations (LmVal) in one of two LDS plane
//     slots; the tile stores u for E and reduces the level's
//     diagnostics;
//   three planes behind, on the tile: a column evaluates, for each of the 3 x
//     3 nodes around it on plane p = a - 3, the post-collision populations
//     whose velocity carries them to this column -- down to plane p - 1, along
//     plane p, up to plane p + 1 -- and adds them to the density and momentum
//     it accumulates for those planes.  Plane p - 1 then has all nineteen: on
//     a wall plane the populations from beyond the wall are the wet-node
//     reconstruction, whose sums are closed forms (below); the column stores
//     the next level's (rho, j).
// A node's staged terms are read from LDS once per neighbour column rather
// than once per population, and nothing but (rho, j, T) in and (rho, j) and U
// out touches memory.  One barrier per plane: the psi slot and the staged
// slot a plane writes were last read before the previous barrier.
//
// Wall planes: the unknown populations of the wet-node reconstruction are f_i
// = f_opp(i) - c_x N_x - c_y N_y with N = half the in-plane momentum.  Summed
// over the five unknown velocities they add the density D of the known
// populations that cross the plane from the lattice side, and cancel the
// momentum exactly: rho' = rho_in + 2 D and j' = 0, the no-slip wall.
//
// The rest population is its closed form w_0 (rho (1 - 3/2 u.u) - 3/2 u.F -
// 3/4 X), which rho less the other populations' sum equals in exact
// arithmetic.

// What LM stages per node of a plane (one LDS slot holds kLmVals planes of
// the region of halo 1): the terms of the node's post-collision populations
// (Eqs. Equilibrium and Guo at tau = 1, with the sigma term) that do not
// depend on the velocity, formed once where the node's force is evaluated.
// For a velocity c = (c_xy, c_z) with a = c_xy . u, b = c_xy . F, A = rho a +
// b, the population is w (e0 + 4.5 (c.u)(rho c.u + c.F) + 3 rho c.u + 1.5 c.F
// + [|c|^2 = 2] s2), and for c_z = +-1 that splits into an even part T0 + Kz
// + s2 and an odd part 4.5 (a B + u_z A) + L, with T0 the value of the c_z =
// 0 bracket.
enum LmVal {
    kRho,
    kUx,
    kUy,
    kUz,
    kFx,
    kFy,
    kB,    // rho u_z + F_z
    kL,    // 3 rho u_z + 3/2 F_z
    kE0,   // rho (1 - 3/2 u.u) - 3/2 u.F
    kS2,   // 3/4 sigma |F_int|^2 / psi^2
    kKz,   // 9/2 u_z (rho u_z + F_z)
    kLmVals
};
// 720 columns in 12 full waves: threads 720 .. 767 hold no column and take
// part in the barriers and the block reduction only
constexpr int kLmColumns = TileE::Threads + TileE::Ring1 + TileE::Ring2;
constexpr int kLmThreads = (kLmColumns + 63) / 64 * 64;

struct Acc4 {
    double r, x, y, z;
};

// a neighbour's staged terms, read from LDS (the fields a velocity group
// does not use are never read: the loads are dead code there)
struct NbVals {
    double rho, ux, uy, uz, Fx, Fy, B, L, e0, s2, Kz;
};
template <int RN>
__device__ __forceinline__ NbVals nb_load(const double (&q)[kLmVals][RN], int m)
{
    return NbVals{q[kRho][m], q[kUx][m], q[kUy][m], q[kUz][m], q[kFx][m], q[kFy][m],
                  q[kB][m],   q[kL][m],  q[kE0][m], q[kS2][m], q[kKz][m]};
}

// the populations a column pulls from its neighbour at offset (OX, OY) on
// plane p: velocity (-OX, -OY, c_z) lands on plane p + c_z, c_z = -1 (lo), 0
// (mid), +1 (hi) where the velocity set has it
template <int OX, int OY>
__device__ __forceinline__ void nb_add(const NbVals &v, Acc4 &lo, Acc4 &mid, Acc4 &hi)
{
    constexpr int cx = -OX, cy = -OY;
    constexpr double w1 = 1.0 / 18.0, w2 = 1.0 / 36.0;
    if (cx == 0 && cy == 0) {
        // rest (its closed form) and the two z-axis velocities
        mid.r += (1.0 / 3.0) * (v.e0 - v.s2);
        const double wE = w1 * (v.e0 + v.Kz), wO = w1 * v.L;
        const double fp = wE + wO, fm = wE - wO;
        hi.r += fp;
        hi.z += fp;
        lo.r += fm;
        lo.z -= fm;
    } else if (cx * cx + cy * cy == 1) {
        // an axis velocity in the plane and the two edges above and below it
        const double a = cx ? cx * v.ux : cy * v.uy;
        const double b = cx ? cx * v.Fx : cy * v.Fy;
        const double A = v.rho * a + b;
        const double T0 = v.e0 + 4.5 * a * A + (3.0 * v.rho * a + 1.5 * b);
        const double f0 = w1 * T0;
        const double wE = w2 * (T0 + (v.Kz + v.s2));
        const double wO = w2 * (4.5 * (a * v.B + v.uz * A) + v.L);
        const double fp = wE + wO, fm = wE - wO;
        mid.r += f0;
        hi.r += fp;
        lo.r += fm;
        if (cx) {
            mid.x += cx * f0;
            hi.x += cx * fp;
            lo.x += cx * fm;
        } else {
            mid.y += cy * f0;
            hi.y += cy * fp;
            lo.y += cy * fm;
        }
        hi.z += fp;
        lo.z -= fm;
    } else {
        // an edge velocity in the plane
        const double a = cx * v.ux + cy * v.uy;
        const double b = cx * v.Fx + cy * v.Fy;
        const double A = v.rho * a + b;
        const double f = w2 * ((v.e0 + v.s2) + 4.5 * a * A + (3.0 * v.rho * a + 1.5 * b));
        mid.r += f;
        mid.x += cx * f;
        mid.y += cy * f;
    }
}

// the pull of a column at region index k from the 3 x 3 neighbours on one
// staged plane, software-pipelined: each neighbour's LDS reads are issued
// before the previous neighbour's arithmetic (the scheduling barriers keep
// the compiler from hoisting all nine neighbours' reads, which would not fit
// in the registers)
template <int RN, int RX>
__device__ __forceinline__ void pull_plane(const double (&q)[kLmVals][RN], int k, Acc4 &lo, Acc4 &mid, Acc4 &hi)
{
    NbVals v0 = nb_load<RN>(q, k - RX - 1);
    __builtin_amdgcn_sched_barrier(0);
    NbVals v1 = nb_load<RN>(q, k - RX);
    nb_add<-1, -1>(v0, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v0 = nb_load<RN>(q, k - RX + 1);
    nb_add<0, -1>(v1, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v1 = nb_load<RN>(q, k - 1);
    nb_add<1, -1>(v0, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v0 = nb_load<RN>(q, k);
    nb_add<-1, 0>(v1, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v1 = nb_load<RN>(q, k + 1);
    nb_add<0, 0>(v0, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v0 = nb_load<RN>(q, k + RX - 1);
    nb_add<1, 0>(v1, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v1 = nb_load<RN>(q, k + RX);
    nb_add<-1, 1>(v0, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    v0 = nb_load<RN>(q, k + RX + 1);
    nb_add<0, 1>(v1, lo, mid, hi);
    __builtin_amdgcn_sched_barrier(0);
    nb_add<1, 1>(v0, lo, mid, hi);
}

template <bool WALLS>
__global__ __launch_bounds__(kLmThreads) void d3q19_march_lm(const double *__restrict__ Min,
                                                            double *__restrict__ Mout,
                                                            const double *__restrict__ Tin, double *__restrict__ U,
                                                            Phys c, Grid3 G, MarchG3 M,
                                                            double *__restrict__ partials,
                                                            StepState *__restrict__ st, int64_t step)
{
    using T = TileE;
    using R2 = T::Region<2>;
    using R1 = T::Region<1>;
    __shared__ double s_psi[4][R2::N];
    __shared__ double s_q[2][kLmVals][R1::N];
    __shared__ double s_red[4 * kLmThreads / 64];
    __shared__ unsigned s_ured[kLmThreads / 64];
    const int t = threadIdx.x;
    const unsigned N = G.N;
    const Seg3 sg = block_segment<T>(M, G.nz);
    const bool tile = t < T::Threads, ring1 = !tile && t < T::Threads + T::Ring1;
    const bool has = t < kLmColumns;
    const bool first = tile || ring1;  // a column of the force stage
    int rx = 2, ry = 2;
    if (tile) {
        rx = t % T::TX + 2;
        ry = t / T::TX + 2;
    } else if (ring1) {
        ring_column<T>(1, 2, t - T::Threads, rx, ry);
    } else if (has) {
        ring_column<T>(2, 2, t - T::Threads - T::Ring1, rx, ry);
    }
    const Col col = make_col(G, sg.x0, sg.y0, rx, ry, 2, R2::RX, has);
    const int r1 = (ry - 1) * R1::RX + (rx - 1);  // index in the region of halo 1 (force-stage columns)
    const bool mine = tile && sg.x0 + rx - 2 < G.nx && sg.y0 + ry - 2 < G.ny;
    const unsigned plane = (unsigned)G.nx * (unsigned)G.ny;
    const unsigned vo = col.n0 * 8u + col.oob;
    const unsigned vj = first ? vo : kOut;   // j is read where the force stage runs
    const unsigned vst = mine ? vo : kOut;   // the tile's lattice columns store
    const double sub = gravity_sub(c.form, st->mean[step & 1], c.rho_v);

    Partial part = {0.0, 0.0, 0.0, 1e300, 0u};
    // rho, j of the column at planes a - 1 (p1) and a - 2 (p2)
    double r_1 = 0.0, x_1 = 0.0, y_1 = 0.0, z_1 = 0.0, r_2 = 0.0, x_2 = 0.0, y_2 = 0.0, z_2 = 0.0;
    // density and momentum pulled so far for planes p - 1, p, p + 1 of the
    // pull of plane p; uplo, upmid: the density of the populations from below
    // (the top wall's reconstruction needs it)
    Acc4 lo = {0.0, 0.0, 0.0, 0.0}, mid = lo;
    double uplo = 0.0, upmid = 0.0;
    // planes z0 - 2 .. z1 + 1 are read, one plane ahead of their use; a read
    // beyond them, or beyond a wall, is an empty range (zeros)
    auto load = [&](int z, double &vr, double &vx, double &vy, double &vz, double &vT) __attribute__((always_inline)) {
        bool beyond;
        const size_t zo = (size_t)plane_of<WALLS>(z, G.nz, beyond) * plane;
        beyond = beyond || z > sg.z1 + 1;
        vr = buf_ld(layer_rsrc(Min + zo, plane, beyond), vo, 0u, 0.0);
        vx = buf_ld(layer_rsrc(Min + N + zo, plane, beyond), vj, 0u, 0.0);
        vy = buf_ld(layer_rsrc(Min + 2 * (size_t)N + zo, plane, beyond), vj, 0u, 0.0);
        vz = buf_ld(layer_rsrc(Min + 3 * (size_t)N + zo, plane, beyond), vj, 0u, 0.0);
        vT = buf_ld(layer_rsrc(Tin + zo, plane, beyond), vo, 0u, 0.0);
    };
    double nr, nx, ny, nzv, nT;
    load(sg.z0 - 2, nr, nx, ny, nzv, nT);
    for (int a = sg.z0 - 2; a <= sg.z1 + 3; ++a) {
        const double ra = nr, xa = nx, ya = ny, za = nzv, Ta = nT;
        load(a + 1, nr, nx, ny, nzv, nT);

        // psi of plane a (nothing beyond a wall)
        {
            bool beyond;
            plane_of<WALLS>(a, G.nz, beyond);
            double Z;
            const double psi = psi_and_Z(c, ra, Ta, Z);
            if (has) s_psi[a & 3][col.r] = beyond ? 0.0 : psi;
        }

        // force stage of plane b = a - 2; the psi planes b - 1 .. b + 1 were
        // written before the previous barrier
        const int b = a - 2;
        if (first && b >= sg.z0 - 1) {  // the first test is per wave, the second uniform
            bool beyond;
            plane_of<WALLS>(b, G.nz, beyond);
            const bool wall = WALLS && (b == 0 || b == G.nz - 1);
            const double psi0 = s_psi[b & 3][col.r];
            // evaluated everywhere and zeroed on wall planes and beyond them
            // (psi there is finite): no branch around the LDS reads
            double sx, sy, sz;
            sc_sum_planes<R2::RX>(s_psi[(b - 1) & 3], s_psi[b & 3], s_psi[(b + 1) & 3], col.r, sx, sy, sz);
            const bool off = wall || beyond;
            const double mg = off ? 0.0 : -c.G * psi0;
            const double Fx = mg * sx, Fy = mg * sy;
            const double Fz = mg * sz + (off ? 0.0 : gravity_force(r_2, sub, c.g));
            const double Xs2 = off ? 0.0 : c.sigma * c.G2 * (sx * sx + sy * sy + sz * sz);  // sigma |F_int|^2 / psi^2
            const double inv = rcp_pos(r_2);
            const double ux = beyond ? 0.0 : (x_2 + 0.5 * Fx) * inv;
            const double uy = beyond ? 0.0 : (y_2 + 0.5 * Fy) * inv;
            const double uz = beyond ? 0.0 : (z_2 + 0.5 * Fz) * inv;
            const double uu = ux * ux + uy * uy + uz * uz;
            const double uF = ux * Fx + uy * Fy + uz * Fz;
            const double Bz = r_2 * uz + Fz;
            double(&q)[kLmVals][R1::N] = s_q[b & 1];
            q[kRho][r1] = r_2;
            q[kUx][r1] = ux;
            q[kUy][r1] = uy;
            q[kUz][r1] = uz;
            q[kFx][r1] = Fx;
            q[kFy][r1] = Fy;
            q[kB][r1] = Bz;
            q[kL][r1] = 3.0 * r_2 * uz + 1.5 * Fz;
            q[kE0][r1] = r_2 * (1.0 - 1.5 * uu) - 1.5 * uF;
            q[kS2][r1] = 0.75 * Xs2;
            q[kKz][r1] = 4.5 * uz * Bz;
            if (tile) {
                const bool live = b >= sg.z0 && b < sg.z1;  // uniform
                const size_t zb = (size_t)(live ? b : sg.z0) * plane;
                buf_st(layer_rsrc(U + zb, plane, !live), vst, 0u, ux);
                buf_st(layer_rsrc(U + N + zb, plane, !live), vst, 0u, uy);
                buf_st(layer_rsrc(U + 2 * (size_t)N + zb, plane, !live), vst, 0u, uz);
                const bool keep = live && mine;
                unsigned fl = 0u;
                if (!(r_2 > 0.0)) fl |= kFlagRho;
                if (c.eos == 0 && c.b_quarter * r_2 >= 1.0) fl |= kFlagEta;
                if (psi0 != psi0) fl |= kFlagPsi;
                if (r_2 != r_2 || uu != uu) fl |= kFlagNaN;
                part.mass_n += keep ? r_2 : 0.0;
                part.umax = keep ? fmax(part.umax, uu) : part.umax;
                part.rmin = keep ? fmin(part.rmin, r_2) : part.rmin;
                part.flags |= keep ? fl : 0u;
            }
        }

        // pull from plane p = a - 3 (written before the previous barrier);
        // plane p - 1 is then complete
        const int p = a - 3;
        if (tile && p >= sg.z0 - 1) {
            const double(&q)[kLmVals][R1::N] = s_q[p & 1];
            Acc4 dlo = {0.0, 0.0, 0.0, 0.0}, hi = dlo;
            pull_plane<R1::N, R1::RX>(q, r1, dlo, mid, hi);
            const int qz = p - 1;
            // on a wall plane nothing has arrived from beyond the wall (its
            // planes hold zeros); selects rather than a branch, which the
            // compiler would turn into a second copy of the march
            const bool wq = WALLS && (qz == 0 || qz == G.nz - 1);
            const double back = WALLS && qz == 0 ? dlo.r : (WALLS && qz == G.nz - 1 ? uplo : 0.0);
            const double rn = (lo.r + dlo.r) + back;
            const double jx = wq ? 0.0 : lo.x + dlo.x, jy = wq ? 0.0 : lo.y + dlo.y, jz = wq ? 0.0 : lo.z + dlo.z;
            const bool live = qz >= sg.z0 && qz < sg.z1;  // uniform
            const size_t zq = (size_t)(live ? qz : sg.z0) * plane;
            buf_st(layer_rsrc(Mout + zq, plane, !live), vst, 0u, rn);
            buf_st(layer_rsrc(Mout + N + zq, plane, !live), vst, 0u, jx);
            buf_st(layer_rsrc(Mout + 2 * (size_t)N + zq, plane, !live), vst, 0u, jy);
            buf_st(layer_rsrc(Mout + 3 * (size_t)N + zq, plane, !live), vst, 0u, jz);
            const bool keep = live && mine;
            part.mass_next += keep ? rn : 0.0;
            part.flags |= (keep && rn != rn) ? kFlagNaN : 0u;
            lo = mid;
            mid = hi;
            uplo = upmid;
            upmid = hi.r;
        }
        r_2 = r_1;
        x_2 = x_1;
        y_2 = y_1;
        z_2 = z_1;
        r_1 = ra;
        x_1 = xa;
        y_1 = ya;
        z_1 = za;
        __syncthreads();
    }
    part = block_reduce<kLmThreads>(part, s_red, s_ured);
    finish_launch<kLmThreads>(part, partials, st, step, (int)((step + 1) & 1), 1.0 / (double)N, s_red, s_ured);
}

template <class T>
MarchG3 march_grid3(int nx, int ny, int nz, int cus, int per_cu = 1)
{
    MarchG3 g;
    g.ntx = (nx + T::TX - 1) / T::TX;
    g.nty = (ny + T::TY - 1) / T::TY;
    const long tiles = (long)g.ntx * g.nty;
    long nseg = ((long)cus * per_cu + tiles - 1) / tiles;
    const long maxseg = nz / 8 > 0 ? nz / 8 : 1;  // segments of at least 8 planes
    if (nseg > maxseg) nseg = maxseg;
    if (nseg < 1) nseg = 1;
    g.nseg = (int)nseg;
    g.nblocks = (int)(tiles * nseg);
    return g;
}

template <class S, bool WALLS>
hipError_t march_t(const LatticeLaunch &L, double *U)
{
    const Grid3 G{L.nx, L.ny, L.nz, (unsigned)((size_t)L.nx * L.ny * L.nz)};
    const MarchG3 M = march_grid3<TileL>(L.nx, L.ny, L.nz, L.resident);
    const MarchG3 ME = march_grid3<TileE>(L.nx, L.ny, L.nz, L.resident, kEBlocksPerCU);
    hipLaunchKernelGGL((d3q19_march_l<S, WALLS>), dim3(M.nblocks), dim3(TileL::Threads), 0, L.stream, (const S *)L.fin,
                       (S *)L.fout, L.Tin, U, L.phys, G, M, L.partials, L.st, L.step, L.rref);
    hipLaunchKernelGGL((d3q19_march_e<WALLS>), dim3(ME.nblocks), dim3(kEThreads), 0, L.stream, L.Tin, L.Tout,
                       (const double *)U, (const double *)U + 3 * (size_t)G.N, L.phys, G, ME);
    return hipGetLastError();
}

// moment state: LM, then E on the same grid of tiles and segments
template <bool WALLS>
hipError_t march_mom_t(const LatticeLaunch &L, double *U)
{
    const Grid3 G{L.nx, L.ny, L.nz, (unsigned)((size_t)L.nx * L.ny * L.nz)};
    const MarchG3 M = march_grid3<TileE>(L.nx, L.ny, L.nz, L.resident, kEBlocksPerCU);
    hipLaunchKernelGGL((d3q19_march_lm<WALLS>), dim3(M.nblocks), dim3(kLmThreads), 0, L.stream,
                       (const double *)L.fin, (double *)L.fout, L.Tin, U, L.phys, G, M, L.partials, L.st, L.step);
    hipLaunchKernelGGL((d3q19_march_e<WALLS>), dim3(M.nblocks), dim3(kEThreads), 0, L.stream, L.Tin, L.Tout,
                       (const double *)U, (const double *)L.fin, L.phys, G, M);
    return hipGetLastError();
}

}  // namespace

// the LBM kernel (L, or LM on E's grid) writes the per-block partials: room
// for the larger grid
int d3q19_march_blocks(int nx, int ny, int nz, int cus)
{
    const int l = march_grid3<TileL>(nx, ny, nz, cus).nblocks;
    const int lm = march_grid3<TileE>(nx, ny, nz, cus, kEBlocksPerCU).nblocks;
    return l > lm ? l : lm;
}

hipError_t d3q19_march_step(const LatticeLaunch &L, double *U)
{
    if (L.moments) return L.walls ? march_mom_t<true>(L, U) : march_mom_t<false>(L, U);
    if (L.fp32) return L.walls ? march_t<float, true>(L, U) : march_t<float, false>(L, U);
    return L.walls ? march_t<double, true>(L, U) : march_t<double, false>(L, U);
}

}  // namespace tplbm
