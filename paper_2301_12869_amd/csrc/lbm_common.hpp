// Device-side building blocks shared by the lattice kernels: physical
// constants, the Carnahan-Starling EOS (Eq. EOS), the Yuan-Schaefer
// pseudopotential (Eq. InteractionPotential) and wavefront/block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tplbm {

// Flags raised by a kernel (same bits as TPLBM_FLAG_* in the public header).
constexpr unsigned kFlagNaN = 1u, kFlagRho = 2u, kFlagEta = 4u, kFlagPsi = 8u;

// Everything a lattice kernel needs about the physics, passed by value.
struct Phys {
    double a, b_quarter, R;   // EOS constants; b_quarter = b/4 so that eta = b_quarter * rho
    double two_over_G;        // 2/G for the pseudopotential radicand
    double G, G2;             // G and G^2 (the sigma term uses |F_int|^2/psi^2 = G^2 |sum w psi c|^2)
    double sigma;
    double kappa_over_cv;     // kappa / c_v
    double R_over_cv;         // R / c_v: (T/(rho c_v)) (dp/dT)_rho = T (R/c_v) Z(eta)
    double g;                 // gravity magnitude (down the wall-normal axis)
    double rho_v;             // gravity form 3: the subtracted vapour density
    double lam[9];            // relaxation rates in moment order (Eq. RelaxationMatrix)
    double sig_e, sig_s;      // sigma / tau_e and sigma / tau_varsigma: the sigma part of (I - Lambda/2) S
    int eos;                  // 0 Carnahan-Starling, 1 ideal lattice gas
    int form;                 // 1: rho g, 2: (rho - <rho>) g, 3: (rho - rho_v) g
};

// Gravity along the wall-normal axis, g > 0 pointing to its first layer
// (Eqs. Gravity_1, Gravity_2, Gravity_3): F_g = -(rho - s) g, where the
// subtracted density s is 0, <rho> or rho_v (-(rho - 0) g is -rho g exactly).
// s is uniform over a launch, so the kernels form it once.
__device__ __forceinline__ double gravity_sub(int form, double mean, double rho_v)
{
    return form == 2 ? mean : (form == 3 ? rho_v : 0.0);
}
__device__ __forceinline__ double gravity_force(double rho, double sub, double g) { return -(rho - sub) * g; }

// Reciprocal of a positive normal double: hardware estimate refined by two
// Newton steps (within about one ulp; no special-case handling, so callers
// pass only finite positive arguments or accept a NaN for anything else).
__device__ __forceinline__ double rcp_pos(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// Square root of a positive normal double by a refined reciprocal square
// root (Goldschmidt-style); zero maps to zero, negative or NaN to NaN.
__device__ __forceinline__ double sqrt_pos(double a)
{
    if (!(a > 0.0)) return a == 0.0 ? 0.0 : __builtin_nan("");
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, a);
    return fma(d, h, g);
}

// Carnahan-Starling compressibility factor Z(eta) = (1+eta+eta^2-eta^3)/(1-eta)^3.
__device__ __forceinline__ double cs_Z(double eta)
{
    const double s = 1.0 - eta;
    const double num = 1.0 + eta * (1.0 + eta * (1.0 - eta));
    return num * rcp_pos(s * s * s);
}

// p_EOS and psi at one node; Zout receives Z(eta) (1 for the ideal gas,
// where the energy equation's compression term vanishes: Zout = 0 then).
__device__ __forceinline__ double psi_and_Z(const Phys &c, double rho, double T, double &Zout)
{
    if (c.eos == 1) {
        Zout = 0.0;
        return 0.0;
    }
    const double Z = cs_Z(c.b_quarter * rho);
    Zout = Z;
    const double p = rho * (c.R * T * Z - c.a * rho);
    // psi = sqrt(2 (p - rho c_s^2) / (G c^2)), c = 1, c_s^2 = 1/3
    return sqrt_pos(c.two_over_G * (p - rho * (1.0 / 3.0)));
}

__device__ __forceinline__ double p_eos(const Phys &c, double rho, double T)
{
    if (c.eos == 1) return rho * (1.0 / 3.0);
    return rho * (c.R * T * cs_Z(c.b_quarter * rho) - c.a * rho);
}

// ---- wavefront (64 lanes) and block reductions ---------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Per-block diagnostic partials: sum of rho at level n, sum of the next
// level's rho (multiplicity-weighted post-collision populations), max |u|^2,
// min rho, flags.
struct Partial {
    double mass_n, mass_next, umax, rmin;
    unsigned flags;
};

// Reduce a Partial over a block of NT threads (NT multiple of 64) in a fixed
// order; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ Partial block_reduce(Partial v, double *scratch /* 4*NT/64 */,
                                                unsigned *uscratch /* NT/64 */)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v.mass_n = wave_sum(v.mass_n);
    v.mass_next = wave_sum(v.mass_next);
    v.umax = wave_max(v.umax);
    v.rmin = wave_min(v.rmin);
    v.flags = wave_or(v.flags);
    if (lane == 0) {
        scratch[w] = v.mass_n;
        scratch[NW + w] = v.mass_next;
        scratch[2 * NW + w] = v.umax;
        scratch[3 * NW + w] = v.rmin;
        uscratch[w] = v.flags;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial r = {0.0, 0.0, 0.0, 1e300, 0u};
        for (int k = 0; k < NW; ++k) {
            r.mass_n += scratch[k];
            r.mass_next += scratch[NW + k];
            r.umax = fmax(r.umax, scratch[2 * NW + k]);
            r.rmin = fmin(r.rmin, scratch[3 * NW + k]);
            r.flags |= uscratch[k];
        }
        v = r;
    }
    return v;
}

// Device-resident step bookkeeping written by the last block of each launch.
struct StepState {
    double mean[2];          // <rho> of the level a launch starts from, by step parity
    double mass;             // sum of rho at the current level
    double max_u, min_rho;   // of the last step's level
    int64_t step;            // completed steps
    int64_t first_bad;       // first level with a flag, -1 if none
    unsigned flags;          // sticky OR of flags
    unsigned counter;        // blocks done in the running launch
};

// Partials are written and read with device-scope atomics so that the last
// block sees every other block's values whatever XCD (and L2) wrote them.
__device__ __forceinline__ void store_partial(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Finish the per-launch reduction: every block calls this once with its
// reduced partial in thread 0.  The last block to arrive sums the partials in
// block order (deterministic), then updates StepState.  `mean_slot` is the
// parity slot that receives <rho> of the next level; `n_nodes` the node count.
template <int NT>
__device__ void finish_launch(const Partial &mine, double *partials, StepState *st, int64_t step,
                              int mean_slot, double inv_nodes, double *scratch,
                              unsigned *uscratch)
{
    __shared__ int s_last;
    const int nblk = gridDim.x;
    if (threadIdx.x == 0) {
        double *p = partials + 5 * (size_t)blockIdx.x;
        store_partial(p + 0, mine.mass_n);
        store_partial(p + 1, mine.mass_next);
        store_partial(p + 2, mine.umax);
        store_partial(p + 3, mine.rmin);
        store_partial(p + 4, (double)mine.flags);
        __threadfence();
        const unsigned prev = atomicAdd(&st->counter, 1u);
        s_last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    Partial acc = {0.0, 0.0, 0.0, 1e300, 0u};
    for (int b = threadIdx.x; b < nblk; b += NT) {
        const double *p = partials + 5 * (size_t)b;
        acc.mass_n += load_partial(p + 0);
        acc.mass_next += load_partial(p + 1);
        acc.umax = fmax(acc.umax, load_partial(p + 2));
        acc.rmin = fmin(acc.rmin, load_partial(p + 3));
        acc.flags |= (unsigned)load_partial(p + 4);
    }
    __syncthreads();
    acc = block_reduce<NT>(acc, scratch, uscratch);
    if (threadIdx.x == 0) {
        st->mean[mean_slot] = acc.mass_next * inv_nodes;
        st->mass = acc.mass_next;
        st->max_u = sqrt(acc.umax);
        st->min_rho = acc.rmin;
        st->step = step + 1;
        if (acc.flags && st->first_bad < 0) st->first_bad = step;
        st->flags |= acc.flags;
        st->counter = 0u;
        __threadfence();
    }
}

}  // namespace tplbm
