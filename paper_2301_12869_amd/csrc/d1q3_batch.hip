// Batched persistent sweep of independent 1-D columns (D1Q3) to steady state.
//
// A column is the x-uniform reduction of the paper's 1-D problem (Sec. IV):
// wall nodes at both ends, liquid below and vapour above, gravity along the
// column.  At tau = 1 the D2Q9 update of an x-uniform field sums, c_y group by
// c_y group, to the D1Q3 update used here: populations f0 (c = 0), f+ and f-
// with weights 2/3, 1/6, 1/6; equilibrium f0 = 2/3 rho (1 - 3/2 u^2),
// f+- = rho/6 (1 +- 3u + 3u^2); Li's forcing reduces to
// F'+- = (uF + sigma X/6)/2 +- F/4, F'0 = -(uF + sigma X/6); the Shan-Chen
// force to -G psi (psi(y+1) - psi(y-1))/2; the isotropic differences of the
// energy equation to central differences; Zou-He at a wall to "the unknown
// population equals the known one" (zero wall velocity).
//
// One workgroup owns one column at a time and takes the next column from a
// device-wide queue when its column converges, diverges or runs out of
// steps, so one launch sweeps the whole batch.  Every thread owns a
// contiguous chunk of at most NPT nodes in registers; values across chunk
// boundaries go through small LDS exchange buffers.  The state held between
// steps is the post-stream level-n populations, as in the oracle.
#include <hip/hip_runtime.h>

#include "batch_internal.hpp"
#include "lbm_common.hpp"

namespace tplbm {

namespace {

// Exchange of chunk-boundary values: each thread publishes the value of its
// first and last node; neighbours read them after a barrier.  Every exchange
// of a step has its own buffer, so one barrier per exchange suffices (a
// buffer is rewritten only in the next step, after several more barriers).
template <int NT>
struct Halo {
    double first[NT];
    double last[NT];
};

template <int NPT>
__device__ __forceinline__ double last_of(const double (&a)[NPT], int npt)
{
    double v = a[0];
#pragma unroll
    for (int k = 1; k < NPT; ++k)
        if (k == npt - 1) v = a[k];
    return v;
}

// Right-hand side of the energy equation with central differences:
// K = -u dT/dy + kappa/(rho c_v) d2T/dy2 - T (R/c_v) Z du/dy.
__device__ __forceinline__ double energy_rhs_1d(const Phys &c, double Tm, double T0, double Tp,
                                                double u0, double divu, double inv_rho, double Z)
{
    const double gy = 0.5 * (Tp - Tm);
    const double lap = (Tp - T0) + (Tm - T0);
    return -u0 * gy + c.kappa_over_cv * inv_rho * lap - T0 * c.R_over_cv * Z * divu;
}

template <int NT, int NPT>
__global__ __launch_bounds__(NT) void d1q3_batch(BatchArgs a, Phys c)
{
    constexpr int NW = NT / 64;
    __shared__ Halo<NT> hpsi, hu, hT, hk, hs;
    __shared__ double red_mass[NW], red_u[NW];
    __shared__ unsigned red_fl[NW];
    __shared__ int s_col;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (;;) {
        if (tid == 0) s_col = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int qi = s_col;
        __syncthreads();
        if (qi >= a.ncols) break;
        const int col = a.order[qi];
        const ColumnDesc d = a.cols[col];
        const int H = d.height;
        const int npt = (H + NT - 1) / NT;  // nodes per thread for this column
        const int y0 = tid * npt;           // first node of this thread
        const double g = d.g;
        const bool form2 = d.form == 2;

        // ---- load: rest populations f = w rho0 (or a previous run's end
        // populations), temperature ----
        double f0[NPT], fp[NPT], fm[NPT], T[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int y = y0 + k;
            const bool own = k < npt && y < H;
            const int64_t i = d.offset + y;
            T[k] = own ? a.T0[i] : 0.0;
            if (a.f_in) {
                f0[k] = own ? a.f_in[i] : 0.0;
                fp[k] = own ? a.f_in[a.nodes + i] : 0.0;
                fm[k] = own ? a.f_in[2 * a.nodes + i] : 0.0;
            } else {
                const double r0 = own ? a.rho0[i] : 0.0;
                f0[k] = 2.0 * r0 / 3.0;
                fp[k] = r0 / 6.0;
                fm[k] = r0 / 6.0;
            }
        }

        int status = 2;
        int64_t n = 0;
        double mass = 0.0, umax = 0.0;
        unsigned fl_seen = 0u;  // flags of every level below the budget so far
        // waves whose first node lies beyond the column own no node: they
        // skip the arithmetic but take part in every barrier (their halo
        // values are never read: the neighbour that would read them is at or
        // beyond the top wall)
        const bool wave_active = wid * 64 * npt < H;
        for (;; ++n) {
            const bool check = n >= a.max_steps || n % a.check_every == 0;
            // ---- phase A: density, momentum, psi; column mass ----
            double rho[NPT], jy[NPT], psi[NPT], Z[NPT];
            double msum = 0.0;
            unsigned fl = 0u;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!wave_active) {
                    rho[k] = jy[k] = psi[k] = Z[k] = 0.0;
                    continue;
                }
                const int y = y0 + k;
                const bool own = k < npt && y < H;
                rho[k] = f0[k] + fp[k] + fm[k];
                jy[k] = fp[k] - fm[k];
                psi[k] = 0.0;
                Z[k] = 0.0;
                if (own) {
                    psi[k] = psi_and_Z(c, rho[k], T[k], Z[k]);
                    msum += rho[k];
                    if (!(rho[k] > 0.0)) fl |= kFlagRho;
                    if (psi[k] != psi[k]) fl |= kFlagPsi;
                    if (c.eos == 0 && c.b_quarter * rho[k] >= 1.0) fl |= kFlagEta;
                }
            }
            hpsi.first[tid] = psi[0];
            hpsi.last[tid] = last_of<NPT>(psi, npt);
            // the column mass: every step for gravity form 2 (its mean enters
            // the force), otherwise only at the check levels (it is reported)
            double tot = 0.0;
            if (form2 || check) {
                msum = wave_active ? wave_sum(msum) : 0.0;
                if (lane == 0) red_mass[wid] = msum;
            }
            __syncthreads();
            if (form2 || check) {
#pragma unroll
                for (int w = 0; w < NW; ++w) tot += red_mass[w];
            }
            const double mean = tot / (double)H;
            const double psiL = tid > 0 ? hpsi.last[tid - 1] : 0.0;
            const double psiR = tid < NT - 1 ? hpsi.first[tid + 1] : 0.0;

            // ---- phase B: force, velocity ----
            double u[NPT], F[NPT], X[NPT], irho[NPT];
            double u2max = 0.0;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!wave_active) {
                    u[k] = F[k] = X[k] = irho[k] = 0.0;
                    continue;
                }
                const int y = y0 + k;
                const bool own = k < npt && y < H;
                const bool wall = y == 0 || y == H - 1;
                const double pm = k > 0 ? psi[k - 1] : psiL;
                const double pp = (k + 1 < npt) ? psi[(k + 1) % NPT] : psiR;
                double Fi = 0.0, Fg = 0.0, sv = 0.0;
                if (own && !wall) {
                    sv = 0.5 * (pp - pm);
                    Fi = -c.G * psi[k] * sv;
                    Fg = gravity_force(rho[k], gravity_sub(d.form, mean, d.rho_v), g);
                }
                F[k] = Fi + Fg;
                X[k] = c.sigma * c.G2 * sv * sv;  // sigma |F_int|^2 / psi^2
                irho[k] = own ? rcp_pos(rho[k]) : 0.0;
                u[k] = own ? (jy[k] + 0.5 * F[k]) * irho[k] : 0.0;
                if (own) u2max = fmax(u2max, u[k] * u[k]);
            }
            // decisions at the check levels, in the oracle's order: a flag at
            // any level below the budget, then the budget, then the steady test
            if (n < a.max_steps) fl_seen |= fl;
            if (check) {
                const double m2w = wave_active ? wave_max(u2max) : 0.0;
                const unsigned flw = wave_active ? wave_or(fl_seen) : 0u;
                if (lane == 0) {
                    red_u[wid] = m2w;
                    red_fl[wid] = flw;
                }
                __syncthreads();
                double m2 = red_u[0];
                unsigned flags = red_fl[0];
#pragma unroll
                for (int w = 1; w < NW; ++w) {
                    m2 = fmax(m2, red_u[w]);
                    flags |= red_fl[w];
                }
                __syncthreads();
                mass = tot;
                umax = sqrt(m2);
                if (flags != 0u) { status = 1; break; }
                if (n >= a.max_steps) { status = 2; break; }
                if (m2 < a.tol * a.tol) { status = 0; break; }
            }
            // exchange u and T boundaries
            hu.first[tid] = u[0];
            hu.last[tid] = last_of<NPT>(u, npt);
            hT.first[tid] = T[0];
            hT.last[tid] = last_of<NPT>(T, npt);
            __syncthreads();
            const double uL = tid > 0 ? hu.last[tid - 1] : 0.0;
            const double uR = tid < NT - 1 ? hu.first[tid + 1] : 0.0;
            const double TL = tid > 0 ? hT.last[tid - 1] : 0.0;
            const double TR = tid < NT - 1 ? hT.first[tid + 1] : 0.0;

            // ---- phase C: first Heun stage ----
            double k1[NPT], divu[NPT];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!wave_active) {
                    k1[k] = divu[k] = 0.0;
                    continue;
                }
                const int y = y0 + k;
                const bool own = k < npt && y < H;
                const bool wall = y == 0 || y == H - 1;
                const double um = k > 0 ? u[k - 1] : uL;
                const double up = (k + 1 < npt) ? u[(k + 1) % NPT] : uR;
                const double Tm = k > 0 ? T[k - 1] : TL;
                const double Tp = (k + 1 < npt) ? T[(k + 1) % NPT] : TR;
                divu[k] = 0.5 * (up - um);
                k1[k] = (own && !wall) ? energy_rhs_1d(c, Tm, T[k], Tp, u[k], divu[k], irho[k], Z[k]) : 0.0;
            }
            hk.first[tid] = k1[0];
            hk.last[tid] = last_of<NPT>(k1, npt);
            __syncthreads();
            const double kL = tid > 0 ? hk.last[tid - 1] : 0.0;
            const double kR = tid < NT - 1 ? hk.first[tid + 1] : 0.0;

            // ---- phase D: second Heun stage, collision ----
            double fs0[NPT], fsp[NPT], fsm[NPT], Tn[NPT];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                Tn[k] = T[k];
                if (!wave_active) {
                    fs0[k] = fsp[k] = fsm[k] = 0.0;
                    continue;
                }
                const int y = y0 + k;
                const bool own = k < npt && y < H;
                const bool wall = y == 0 || y == H - 1;
                if (own && !wall) {
                    const double Tm = (k > 0 ? T[k - 1] : TL) + (k > 0 ? k1[k - 1] : kL);
                    const double Tp = ((k + 1 < npt) ? T[(k + 1) % NPT] : TR) +
                                      ((k + 1 < npt) ? k1[(k + 1) % NPT] : kR);
                    const double k2 = energy_rhs_1d(c, Tm, T[k] + k1[k], Tp, u[k], divu[k], irho[k], Z[k]);
                    Tn[k] = T[k] + 0.5 * (k1[k] + k2);
                }
                // tau = 1: f* = f_eq + F'; the rest population closes the mass
                const double r = rho[k], uu = u[k], Fk = F[k];
                const double q = uu * Fk + X[k] * (1.0 / 6.0);
                const double r6 = r / 6.0;
                const double e = r6 * (1.0 + 3.0 * uu * uu) + 0.5 * q;
                const double o = r6 * 3.0 * uu + 0.25 * Fk;
                fsp[k] = e + o;
                fsm[k] = e - o;
                fs0[k] = r - (fsp[k] + fsm[k]);
            }
            // ---- streaming with the Zou-He walls ----
            hs.first[tid] = fsm[0];               // moves to the previous node
            hs.last[tid] = last_of<NPT>(fsp, npt);  // moves to the next node
            __syncthreads();
            const double inP = tid > 0 ? hs.last[tid - 1] : 0.0;
            const double inM = tid < NT - 1 ? hs.first[tid + 1] : 0.0;
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int y = y0 + k;
                T[k] = Tn[k];
                f0[k] = fs0[k];
                fp[k] = k > 0 ? fsp[k - 1] : inP;
                fm[k] = (k + 1 < npt) ? fsm[(k + 1) % NPT] : inM;
                if (y == 0) fp[k] = fm[k];      // bottom wall: unknown f+ = f-
                if (y == H - 1) fm[k] = fp[k];  // top wall: unknown f- = f+
            }
        }

        // ---- outputs of the final level: rho, T, populations; per-column
        // result ----
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int y = y0 + k;
            if (k < npt && y < H) {
                const int64_t i = d.offset + y;
                a.rho_out[i] = f0[k] + fp[k] + fm[k];
                a.T_out[i] = T[k];
                if (a.f_out) {
                    a.f_out[i] = f0[k];
                    a.f_out[a.nodes + i] = fp[k];
                    a.f_out[2 * a.nodes + i] = fm[k];
                }
            }
        }
        if (tid == 0) {
            ColumnResult res;
            res.steps = n;
            res.status = status;
            res.pad = 0;
            res.mass = mass;
            res.max_u = umax;
            a.results[col] = res;
        }
        __syncthreads();
    }
}

template <int NT, int NPT>
hipError_t launch(const BatchArgs &a, const Phys &c, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((d1q3_batch<NT, NPT>), dim3(grid), dim3(NT), 0, s, a, c);
    return hipGetLastError();
}

}  // namespace

const BatchShape kBatchShapes[] = {{256, 8}, {512, 4}, {1024, 2}, {128, 16}};
const int kNumBatchShapes = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);

hipError_t d1q3_batch_launch(int shape, const BatchArgs &a, const Phys &c, int grid, hipStream_t s)
{
    switch (shape) {
    case 0: return launch<256, 8>(a, c, grid, s);
    case 1: return launch<512, 4>(a, c, grid, s);
    case 2: return launch<1024, 2>(a, c, grid, s);
    case 3: return launch<128, 16>(a, c, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tplbm

namespace tplbm {
hipError_t d1q3_batch_occupancy(int shape, int *blocks_per_cu)
{
    switch (shape) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, d1q3_batch<256, 8>, 256, 0);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, d1q3_batch<512, 4>, 512, 0);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, d1q3_batch<1024, 2>, 1024, 0);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, d1q3_batch<128, 16>, 128, 0);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace tplbm
