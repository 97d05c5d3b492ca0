// D3Q19 building blocks shared by the pass kernels (d3q19.hip) and the
// z-marching update (d3q19_march.hip): the velocity set and its weights,
// and population storage (FP64, or FP32 deviations from w_i rho_ref).
#pragma once
#include <hip/hip_runtime.h>

#include "lbm_common.hpp"
#include "lbm_internal.hpp"

namespace tplbm {
namespace d3 {

// Lattice shape: nx x ny x nz nodes, N of them (indices fit 32 bits).
struct Grid3 {
    int nx, ny, nz;
    unsigned N;
};

// velocity set: 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 edges (the table
// the host uses to lay out initial states, kD3Q19* in lbm_internal.hpp)
struct V3 {
    int x, y, z;
};
__host__ __device__ constexpr V3 vel(int i) { return V3{kD3Q19x[i], kD3Q19y[i], kD3Q19z[i]}; }
__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
// c . (a, b, c) over the nonzero components of c only, in x, y, z order.  In
// the unrolled loops c is a compile-time constant, so a zero component costs
// neither a load nor a multiply-add; the result equals the full sum (the
// skipped terms are signed zeros).
__device__ __forceinline__ double cdot(const V3 v, double a, double b, double c)
{
    double s = 0.0;
    bool any = false;
    if (v.x) { s = v.x * a; any = true; }
    if (v.y) { s = any ? s + v.y * b : v.y * b; any = true; }
    if (v.z) { s = any ? s + v.z * c : v.z * c; any = true; }
    return s;
}

// opposite velocity
__host__ __device__ constexpr int opp(int i)
{
    constexpr int o[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    return o[i];
}

template <class S>
struct Pop;
// ld: the population value at index i (wr = w_i rho_ref for FP32
// deviations); st: store v, returning the value as stored (rounded); raw and
// val split ld into the memory access and the conversion.
template <>
struct Pop<double> {
    __device__ static __forceinline__ double raw(const double *p, size_t i) { return p[i]; }
    __device__ static __forceinline__ double val(double r, double) { return r; }
    __device__ static __forceinline__ double ld(const double *p, size_t i, double) { return p[i]; }
    __device__ static __forceinline__ double st(double *p, size_t i, double v, double)
    {
        p[i] = v;
        return v;
    }
};
template <>
struct Pop<float> {
    __device__ static __forceinline__ float raw(const float *p, size_t i) { return p[i]; }
    __device__ static __forceinline__ double val(float r, double wr) { return wr + (double)r; }
    __device__ static __forceinline__ double ld(const float *p, size_t i, double wr) { return wr + (double)p[i]; }
    __device__ static __forceinline__ double st(float *p, size_t i, double v, double wr)
    {
        const float d = (float)(v - wr);
        p[i] = d;
        return wr + (double)d;
    }
};

}  // namespace d3
}  // namespace tplbm
