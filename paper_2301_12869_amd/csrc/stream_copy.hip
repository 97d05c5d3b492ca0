// Streaming device-to-device copy with 16-byte vector loads and stores: the
// HBM rate a bandwidth-bound kernel of this library can reach on this GPU,
// measured by the benchmark beside the lattice kernels (which are measured
// against the 8 TB/s datasheet peak).
//
// Shape: one 16-byte vector per thread and as many workgroups as that takes
// (a grid-stride loop only beyond the grid limit).  Measured on one MI355X
// with a 1 GiB buffer, this moves 6.2 TB/s (read + write); the same loop with
// a persistent grid of 4-32 workgroups per compute unit and 1-8 vectors per
// thread moved 4.0-5.7 TB/s, and non-temporal accesses did not help.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tplbm.h"

namespace {

constexpr int kCopyThreads = 256;
constexpr size_t kMaxGrid = 1u << 30;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte vector

__global__ __launch_bounds__(kCopyThreads) void stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                            size_t nvec, const unsigned char *__restrict__ src_tail,
                                                            unsigned char *__restrict__ dst_tail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * kCopyThreads;
    for (size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; i < nvec; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0)
        for (size_t t = threadIdx.x; t < ntail; t += kCopyThreads) dst_tail[t] = src_tail[t];
}

}  // namespace

extern "C" int tplbm_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *hip_stream)
{
    if (bytes == 0) return TPLBM_OK;
    if (!dev_src || !dev_dst) return TPLBM_EINVAL;
    if (((uintptr_t)dev_src & 15) != 0 || ((uintptr_t)dev_dst & 15) != 0) return TPLBM_EINVAL;
    const size_t nvec = bytes / 16, ntail = bytes - nvec * 16;
    size_t grid = (nvec + kCopyThreads - 1) / kCopyThreads;
    grid = grid < 1 ? 1 : (grid > kMaxGrid ? kMaxGrid : grid);
    hipLaunchKernelGGL(stream_copy, dim3((unsigned)grid), dim3(kCopyThreads), 0, (hipStream_t)hip_stream,
                       (const u32x4 *)dev_src, (u32x4 *)dev_dst, nvec,
                       (const unsigned char *)dev_src + nvec * 16, (unsigned char *)dev_dst + nvec * 16, ntail);
    return hipGetLastError() == hipSuccess ? TPLBM_OK : TPLBM_EHIP;
}
