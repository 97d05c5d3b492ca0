// D3Q19 thermal pseudopotential update for gfx950 (every relaxation time 1,
// where the MRT collision is the BGK one): a 3-D extension of the paper's
// D2Q9 method, walls on the z layers, periodic in x and y.
//
// Velocities: rest, 6 axis neighbours (w = 1/18), 12 edge neighbours
// (w = 1/36).  Shan-Chen weights w(1) = 1/6, w(2) = 1/12 (sum w c_a c_b =
// delta_ab, as for the paper's D2Q9 weights).  Forcing at tau = 1: half of
// Guo's term plus the isotropic sigma term w_i (|c_i|^2 - 1)(3/4) sigma X',
// the D2Q9 sigma term of Li's scheme written without the 2-D moment basis.
//
// This file holds the readout passes.  Both states (the populations, FP32
// deviations or FP64, and the FP64 moment state) are advanced by the
// z-marching kernels of d3q19_march.hip; a readout rebuilds the level's
// fields here:
//   A: pull-stream with Zou-He wall reconstruction, rho, j, psi -> M (the
//      moment state is M itself, whose psi plane the readout fills)
//   B: Shan-Chen force (zero at walls), gravity, u = (j + F/2)/rho, and
//      sigma |F_int|^2 / psi^2                               -> U (u, F, X)
// and the readout kernel forms the requested field from M, U and T.
#include <hip/hip_runtime.h>

#include "d3q19_common.hpp"
#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {

using namespace d3;

// Lattice shape and the row a block works on.  A block owns whole x-rows
// (fixed y, z); the nine rows at y + dy, z + dz (dy, dz in {-1, 0, 1}) have
// their first node's index computed once per row, so a neighbour index is a
// row offset plus a wrapped x: 32-bit, no division per node.  On z-walls the
// rows beyond the lattice are clamped to the wall row (only pulls use them,
// and those populations are reconstructed).

struct Rows {
    unsigned b[3][3];  // [dz + 1][dy + 1]
    __device__ __forceinline__ unsigned at(int dx_wrapped_x, int dy, int dz) const
    {
        return b[dz + 1][dy + 1] + (unsigned)dx_wrapped_x;
    }
};

template <bool WALLS>
__device__ __forceinline__ Rows row_bases(const Grid3 &G, int y, int z)
{
    Rows r;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        int zz = z + dz;
        if (WALLS) zz = zz < 0 ? 0 : (zz >= G.nz ? G.nz - 1 : zz);
        else zz = zz < 0 ? zz + G.nz : (zz >= G.nz ? zz - G.nz : zz);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            int yy = y + dy;
            yy = yy < 0 ? yy + G.ny : (yy >= G.ny ? yy - G.ny : yy);
            r.b[dz + 1][dy + 1] = ((unsigned)zz * (unsigned)G.ny + (unsigned)yy) * (unsigned)G.nx;
        }
    }
    return r;
}

__device__ __forceinline__ int wrap_x(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// Rows of this block.  Blocks are dispatched round-robin over the 8 XCDs;
// with a grid that is a multiple of 8, XCD k takes the k-th contiguous
// eighth of the rows (z-slabs), so the neighbouring rows a stencil reads
// were mostly brought into that XCD's L2 by its own blocks.
struct RowIter {
    int first, end, step;
};
__device__ __forceinline__ RowIter row_iter(int rows)
{
    RowIter it;
    const int nb = gridDim.x;
    if ((nb & 7) == 0 && rows >= nb) {
        const int per = nb >> 3, chunk = (rows + 7) >> 3;
        const int r0 = (blockIdx.x & 7) * chunk;
        it.first = r0 + (blockIdx.x >> 3);
        it.end = min(rows, r0 + chunk);
        it.step = per;
    } else {
        it.first = blockIdx.x;
        it.end = rows;
        it.step = nb;
    }
    return it;
}

// x-neighbours x - 1, x, x + 1 (periodic)
struct Xs {
    int v[3];
};
__device__ __forceinline__ Xs xs_of(int x, int nx)
{
    Xs q;
    q.v[0] = wrap_x(x - 1, nx);
    q.v[1] = x;
    q.v[2] = wrap_x(x + 1, nx);
    return q;
}

// ---- pass A: pull, Zou-He, moments, psi ----------------------------------
template <class S, bool WALLS>
__global__ __launch_bounds__(256) void d3q19_pass_a(const S *__restrict__ fin, const double *__restrict__ Tin,
                                                    double *__restrict__ M, Phys c, Grid3 G,
                                                    const double *__restrict__ rref)
{
    const unsigned N = G.N;
    const int rows = G.ny * G.nz;
    const RowIter it = row_iter(rows);
    for (int row = it.first; row < it.end; row += it.step) {
        const int y = row % G.ny, z = row / G.ny;
        const Rows R = row_bases<WALLS>(G, y, z);
        // FP32: reference densities of the planes the pulled values are
        // stored in (z - c_z; beyond a wall the plane itself, whose values
        // are then reconstructed)
        double rz[3] = {0.0, 0.0, 0.0};
        if (sizeof(S) == 4) {
            int zm = z - 1, zp = z + 1;
            if (WALLS) {
                zm = zm < 0 ? 0 : zm;
                zp = zp >= G.nz ? G.nz - 1 : zp;
            } else {
                zm = zm < 0 ? zm + G.nz : zm;
                zp = zp >= G.nz ? zp - G.nz : zp;
            }
            rz[0] = rref[zm];
            rz[1] = rref[z];
            rz[2] = rref[zp];
        }
        for (int x = threadIdx.x; x < G.nx; x += blockDim.x) {
            const unsigned n = R.at(x, 0, 0);
            const Xs X = xs_of(x, G.nx);
            double f[19];
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const V3 v = vel(i);
                f[i] = Pop<S>::ld(fin, (size_t)i * N + R.at(X.v[1 - v.x], -v.y, -v.z), wgt(i) * rz[1 - v.z]);
            }
            if (WALLS && (z == 0 || z == G.nz - 1)) {
                // zero-velocity wet-node reconstruction of the populations that
                // come from beyond the wall, with transverse momentum corrections
                const int s = z == 0 ? 1 : -1;
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
            double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const V3 v = vel(i);
                rho += f[i];
                if (v.x) jx += v.x * f[i];
                if (v.y) jy += v.y * f[i];
                if (v.z) jz += v.z * f[i];
            }
            double Z;
            const double psi = psi_and_Z(c, rho, Tin[n], Z);
            M[n] = rho;
            M[N + n] = jx;
            M[2 * (size_t)N + n] = jy;
            M[3 * (size_t)N + n] = jz;
            M[4 * (size_t)N + n] = psi;
        }
    }
}

// ---- tiles for the stencil passes -------------------------------------------
// Pass B evaluates 18-neighbour stencils.  A block takes a tile of
// TX x TY x TZ nodes, stages the stencil fields of the tile plus a one-node
// halo ((TX + 2) x (TY + 2) x (TZ + 2), the region) in LDS once, and
// evaluates every stencil from there.  Tiles are walked persistently; XCD k
// takes the k-th contiguous eighth of them (z-slabs), as for the rows of
// pass A.
template <int TX_, int TY_, int TZ_>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_, TZ = TZ_;
    static constexpr int RX = TX + 2, RY = TY + 2, RZ = TZ + 2;
    static constexpr int Region = RX * RY * RZ, Nodes = TX * TY * TZ;
    __host__ __device__ static int count(int nx, int ny, int nz)
    {
        return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + TZ - 1) / TZ);
    }
};
// Pass B stages one field (the region of a 64 x 8 x 4 tile: 66 x 10 x 6
// nodes, 31.7 KB).
using TileBD = TileShape<64, 8, 4>;
constexpr int kStencilThreads = 512;

struct TileIter {
    int first, end, step;
};
__device__ __forceinline__ TileIter tile_iter(int ntiles)
{
    TileIter it;
    const int nb = gridDim.x;
    if ((nb & 7) == 0 && ntiles >= nb) {
        const int chunk = (ntiles + 7) >> 3;
        const int t0 = (blockIdx.x & 7) * chunk;
        it.first = t0 + (blockIdx.x >> 3);
        it.end = min(ntiles, t0 + chunk);
        it.step = nb >> 3;
    } else {
        it.first = blockIdx.x;
        it.end = ntiles;
        it.step = nb;
    }
    return it;
}

struct Tile3 {
    int x0, y0, z0;
};
template <class Sh>
__device__ __forceinline__ Tile3 tile_origin(const Grid3 &G, int t)
{
    const int tx = (G.nx + Sh::TX - 1) / Sh::TX, ty = (G.ny + Sh::TY - 1) / Sh::TY;
    Tile3 o;
    o.x0 = (t % tx) * Sh::TX;
    o.y0 = ((t / tx) % ty) * Sh::TY;
    o.z0 = (t / (tx * ty)) * Sh::TZ;
    return o;
}

__device__ __forceinline__ int periodic(int v, int n) { return v < 0 ? n - 1 : (v >= n ? v % n : v); }

// global index of region node r (periodic x, y; z periodic or clamped at
// walls -- clamped values are never used by a stencil)
template <bool WALLS, class Sh>
__device__ __forceinline__ unsigned region_index(const Grid3 &G, const Tile3 &o, int r)
{
    const int rx = r % Sh::RX, ry = (r / Sh::RX) % Sh::RY, rz = r / (Sh::RX * Sh::RY);
    const int x = periodic(o.x0 + rx - 1, G.nx), y = periodic(o.y0 + ry - 1, G.ny);
    int z = o.z0 + rz - 1;
    if (WALLS) z = z < 0 ? 0 : (z >= G.nz ? G.nz - 1 : z);
    else z = periodic(z, G.nz);
    return ((unsigned)z * (unsigned)G.ny + (unsigned)y) * (unsigned)G.nx + (unsigned)x;
}

// region index of the neighbour (dx, dy, dz) of tile node (tx, ty, tz)
template <class Sh>
__device__ __forceinline__ int rnb(int tx, int ty, int tz, int dx, int dy, int dz)
{
    return ((tz + 1 + dz) * Sh::RY + (ty + 1 + dy)) * Sh::RX + (tx + 1 + dx);
}

// Shan-Chen sum s = sum_i w(|c_i|^2) psi(x + c_i) c_i, w(1) = 1/6, w(2) = 1/12
template <class Sh>
__device__ __forceinline__ void sc_sum(const double *__restrict__ sp, int tx, int ty, int tz, double &sx,
                                       double &sy, double &sz)
{
    sx = sy = sz = 0.0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const V3 v = vel(i);
        const double w = i < 7 ? 1.0 / 6.0 : 1.0 / 12.0;
        const double p = sp[rnb<Sh>(tx, ty, tz, v.x, v.y, v.z)];
        if (v.x) sx += w * v.x * p;
        if (v.y) sy += w * v.y * p;
        if (v.z) sz += w * v.z * p;
    }
}

// ---- pass B: force and velocity --------------------------------------------
template <bool WALLS>
__global__ __launch_bounds__(kStencilThreads) void d3q19_pass_b(const double *__restrict__ M, double *__restrict__ U,
                                                                Phys c, Grid3 G, const StepState *__restrict__ st,
                                                                int slot)
{
    using Sh = TileBD;
    __shared__ double s_psi[Sh::Region];
    const unsigned N = G.N;
    const double mean = st->mean[slot];
    const int ntiles = Sh::count(G.nx, G.ny, G.nz);
    const TileIter it = tile_iter(ntiles);
    for (int t = it.first; t < it.end; t += it.step) {
        const Tile3 o = tile_origin<Sh>(G, t);
        __syncthreads();
        for (int r = threadIdx.x; r < Sh::Region; r += kStencilThreads)
            s_psi[r] = M[4 * (size_t)N + region_index<WALLS, Sh>(G, o, r)];
        __syncthreads();
        for (int k = threadIdx.x; k < Sh::Nodes; k += kStencilThreads) {
            const int tx = k % Sh::TX, ty = (k / Sh::TX) % Sh::TY, tz = k / (Sh::TX * Sh::TY);
            const int x = o.x0 + tx, y = o.y0 + ty, z = o.z0 + tz;
            if (x >= G.nx || y >= G.ny || z >= G.nz) continue;
            const unsigned n = ((unsigned)z * (unsigned)G.ny + (unsigned)y) * (unsigned)G.nx + (unsigned)x;
            const double rho = M[n];
            double Fx = 0.0, Fy = 0.0, Fz = 0.0, Xs2 = 0.0;
            if (!(WALLS && (z == 0 || z == G.nz - 1))) {
                double sx, sy, sz;
                sc_sum<Sh>(s_psi, tx, ty, tz, sx, sy, sz);
                const double mg = -c.G * s_psi[rnb<Sh>(tx, ty, tz, 0, 0, 0)];
                Fx = mg * sx;
                Fy = mg * sy;
                Fz = mg * sz + gravity_force(rho, gravity_sub(c.form, mean, c.rho_v), c.g);
                Xs2 = c.sigma * c.G2 * (sx * sx + sy * sy + sz * sz);  // sigma |F_int|^2 / psi^2
            }
            const double inv = rcp_pos(rho);
            U[n] = (M[N + n] + 0.5 * Fx) * inv;
            U[N + n] = (M[2 * (size_t)N + n] + 0.5 * Fy) * inv;
            U[2 * (size_t)N + n] = (M[3 * (size_t)N + n] + 0.5 * Fz) * inv;
            U[3 * (size_t)N + n] = Fx;
            U[4 * (size_t)N + n] = Fy;
            U[5 * (size_t)N + n] = Fz;
            U[6 * (size_t)N + n] = Xs2;
        }
    }
}

// psi of level 0 for the moment state (rho and j come from the host)
__global__ void d3q19_psi_init(double *__restrict__ M, const double *__restrict__ Tin, Phys c, unsigned N)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
        double Z;
        M[4 * (size_t)N + n] = psi_and_Z(c, M[n], Tin[n], Z);
    }
}

// ---- readout: from M and U of the current level -------------------------------
template <bool WALLS>
__global__ void d3q19_readout(const double *__restrict__ M, const double *__restrict__ U,
                              const double *__restrict__ Tin, Phys c, Grid3 G, int field,
                              double *__restrict__ out)
{
    const unsigned N = G.N;
    const int rows = G.ny * G.nz;
    const RowIter it = row_iter(rows);
    for (int row = it.first; row < it.end; row += it.step) {
        const int y = row % G.ny, z = row / G.ny;
        const Rows R = row_bases<WALLS>(G, y, z);
        for (int x = threadIdx.x; x < G.nx; x += blockDim.x) {
            const unsigned n = R.at(x, 0, 0);
            const double r = M[n];
            double v = 0.0;
            if (field == 0) v = r;
            else if (field == 1) v = U[n];
            else if (field == 2) v = U[N + n];
            else if (field == 3) v = U[2 * (size_t)N + n];
            else if (field == 4) v = Tin[n];
            else {
                const double pe = p_eos(c, r, Tin[n]);
                v = pe;
                if (field == 6 && !(WALLS && (z == 0 || z == G.nz - 1))) {
                    const double *psi = M + 4 * (size_t)N;
                    const Xs X = xs_of(x, G.nx);
                    const double p0 = psi[n];
                    const double pxp = psi[R.at(X.v[2], 0, 0)], pxm = psi[R.at(X.v[0], 0, 0)];
                    const double pyp = psi[R.at(x, 1, 0)], pym = psi[R.at(x, -1, 0)];
                    const double pzp = psi[R.at(x, 0, 1)], pzm = psi[R.at(x, 0, -1)];
                    const double dx = 0.5 * (pxp - pxm), dy = 0.5 * (pyp - pym), dz = 0.5 * (pzp - pzm);
                    const double lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - 6.0 * p0;
                    const double dzz = (pzp + pzm) - 2.0 * p0;
                    v = pe + c.sigma * c.G2 * (1.0 / 6.0) * (dx * dx + dy * dy + dz * dz) +
                        c.G * (1.0 / 12.0) * p0 * lap + c.G * (1.0 / 6.0) * p0 * dzz;
                }
            }
            out[n] = v;
        }
    }
}

// one block per x-row (fixed y, z), at most 8 resident blocks per compute unit
int grid_rows(int ny, int nz, int cus)
{
    const long rows = (long)ny * nz;
    const long cap = (long)cus * 8;
    return (int)(rows < cap ? rows : cap);
}

// one block per tile, at most 4 resident blocks per compute unit (LDS)
template <class Sh>
int grid_tiles(int nx, int ny, int nz, int cus)
{
    const long t = Sh::count(nx, ny, nz);
    const long cap = (long)cus * 4;
    return (int)(t < cap ? t : cap);
}

}  // namespace

// the grid that writes per-block partials (the z-marching LBM kernel)
int d3q19_num_blocks(int nx, int ny, int nz, int cus) { return d3q19_march_blocks(nx, ny, nz, cus); }

hipError_t d3q19_launch_step(const LatticeLaunch &L, double *U) { return d3q19_march_step(L, U); }

hipError_t d3q19_launch_psi_init(const LatticeLaunch &L, double *M)
{
    const unsigned N = (unsigned)((size_t)L.nx * L.ny * L.nz);
    const int threads = 256;
    const int blocks = (int)((N + threads - 1) / threads < 65535 ? (N + threads - 1) / threads : 65535);
    hipLaunchKernelGGL(d3q19_psi_init, dim3(blocks), dim3(threads), 0, L.stream, M, L.Tin, L.phys, N);
    return hipGetLastError();
}

hipError_t d3q19_launch_readout(const LatticeLaunch &L, int field, double *M, double *U, double *out)
{
    const Grid3 G{L.nx, L.ny, L.nz, (unsigned)((size_t)L.nx * L.ny * L.nz)};
    const int g = grid_rows(L.ny, L.nz, L.resident);
    if (L.moments) {
        // the state is M itself; its psi plane is the readout's to fill
        M = (double *)L.fin;
        const hipError_t e = d3q19_launch_psi_init(L, M);
        if (e != hipSuccess) return e;
    } else if (L.fp32) {
        if (L.walls)
            hipLaunchKernelGGL((d3q19_pass_a<float, true>), dim3(g), dim3(256), 0, L.stream, (const float *)L.fin, L.Tin, M, L.phys, G, L.rref);
        else
            hipLaunchKernelGGL((d3q19_pass_a<float, false>), dim3(g), dim3(256), 0, L.stream, (const float *)L.fin, L.Tin, M, L.phys, G, L.rref);
    } else {
        if (L.walls)
            hipLaunchKernelGGL((d3q19_pass_a<double, true>), dim3(g), dim3(256), 0, L.stream, (const double *)L.fin, L.Tin, M, L.phys, G, L.rref);
        else
            hipLaunchKernelGGL((d3q19_pass_a<double, false>), dim3(g), dim3(256), 0, L.stream, (const double *)L.fin, L.Tin, M, L.phys, G, L.rref);
    }
    const int gT = grid_tiles<TileBD>(L.nx, L.ny, L.nz, L.resident);
    if (L.walls) {
        hipLaunchKernelGGL((d3q19_pass_b<true>), dim3(gT), dim3(kStencilThreads), 0, L.stream, M, U, L.phys, G, L.st, (int)(L.step & 1));
        hipLaunchKernelGGL((d3q19_readout<true>), dim3(g), dim3(256), 0, L.stream, M, U, L.Tin, L.phys, G, field, out);
    } else {
        hipLaunchKernelGGL((d3q19_pass_b<false>), dim3(gT), dim3(kStencilThreads), 0, L.stream, M, U, L.phys, G, L.st, (int)(L.step & 1));
        hipLaunchKernelGGL((d3q19_readout<false>), dim3(g), dim3(256), 0, L.stream, M, U, L.Tin, L.phys, G, field, out);
    }
    return hipGetLastError();
}

}  // namespace tplbm
