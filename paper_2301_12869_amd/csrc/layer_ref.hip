// Per-layer reference densities of FP32-deviation storage.
//
// An FP32 lattice stores each post-collision population as the deviation
// d_i = f_i - w_i rho_ref(layer) from the equilibrium at rest of a reference
// density of the wall-normal layer it is stored in (a row in 2-D, a plane in
// 3-D).  Re-centring sets every layer's reference to the layer's current
// mean density (the sum of its stored post-collision populations, which
// equals its density at the level they stream to, divided by its node
// count) and re-encodes the layer's deviations around it, so that they stay
// small where the phases and the interface sit now.  The populations change
// by at most one FP32 rounding of the new deviation; the level's <rho> is
// then recomputed from the re-encoded values with the same wall
// multiplicities the step kernels use.
#include <hip/hip_runtime.h>

#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {

namespace {

constexpr int kLayerThreads = 256;

__device__ __forceinline__ double block_sum_256(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// One block per layer: the layer's mean density, the re-encoding, and the
// layer's share of the next level's mass (multiplicity-weighted).
__global__ __launch_bounds__(kLayerThreads) void recentre_layers(float *__restrict__ f, double *__restrict__ rref,
                                                                 double *__restrict__ lmass, size_t N,
                                                                 int lnodes, int nl, LayerSet q, int walls)
{
    __shared__ double red[kLayerThreads / 64];
    const int layer = blockIdx.x;
    const size_t base = (size_t)layer * (size_t)lnodes;
    const double r_old = rref[layer];
    double s = 0.0;
    for (int k = threadIdx.x; k < lnodes; k += kLayerThreads) {
        double m = 0.0;
        for (int i = 0; i < q.Q; ++i) m += q.w[i] * r_old + (double)f[(size_t)i * N + base + k];
        s += m;
    }
    const double r_new = block_sum_256(s, red) / (double)lnodes;
    double nm = 0.0, down = 0.0, up = 0.0;
    for (int k = threadIdx.x; k < lnodes; k += kLayerThreads) {
        for (int i = 0; i < q.Q; ++i) {
            const size_t idx = (size_t)i * N + base + k;
            const double v = q.w[i] * r_old + (double)f[idx];
            const float d = (float)(v - q.w[i] * r_new);
            f[idx] = d;
            const double vn = q.w[i] * r_new + (double)d;  // what the next step reads
            nm += vn;
            if (q.cn[i] < 0) down += vn;
            if (q.cn[i] > 0) up += vn;
        }
    }
    nm = block_sum_256(nm, red);
    down = block_sum_256(down, red);
    up = block_sum_256(up, red);
    if (threadIdx.x == 0) {
        // a population moving into a wall layer is counted twice by that
        // wall's reconstruction, one leaving through a wall not at all
        if (walls) {
            if (layer == 0) nm -= down;
            if (layer == 1) nm += down;
            if (layer == nl - 2) nm += up;
            if (layer == nl - 1) nm -= up;
        }
        lmass[layer] = nm;
        rref[layer] = r_new;
    }
}

// <rho> and mass of the level from the layers' shares, in layer order.
__global__ __launch_bounds__(1024) void recentre_finish(const double *__restrict__ lmass, int nl, double inv_nodes,
                                                        StepState *__restrict__ st, int slot)
{
    __shared__ double red[16];
    double s = 0.0;
    const int per = (nl + 1023) / 1024;
    const int k0 = threadIdx.x * per, k1 = min(k0 + per, nl);
    for (int k = k0; k < k1; ++k) s += lmass[k];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k];
        st->mean[slot] = t * inv_nodes;
        st->mass = t;
    }
}

}  // namespace

hipError_t recentre_layers_launch(float *f, double *rref, double *lmass, size_t N, int lnodes, int nlayers,
                                  const LayerSet &q, bool walls, StepState *st, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(recentre_layers, dim3(nlayers), dim3(kLayerThreads), 0, s, f, rref, lmass, N, lnodes,
                       nlayers, q, walls ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(recentre_finish, dim3(1), dim3(1024), 0, s, (const double *)lmass, nlayers,
                       1.0 / (double)N, st, slot);
    return hipGetLastError();
}

}  // namespace tplbm
