// Allocation-free variant of the batched column sweep (tplbm_batch_run_noalloc
// in include/tplbm.h) for callers that cannot allocate device memory.
//
// The caller passes the inputs (column descriptions, initial densities and
// temperatures) and the outputs (end densities, temperatures, per-column
// results).  What the sweep needs beyond them -- the device copy of the
// column descriptions, their node offsets, the processing order and the
// work-queue counter of the persistent launch -- lives in one file-scope
// device array per GPU.  Host code never uses the array's name as an
// address: the device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <mutex>

#include "../../include/tplbm.h"
#include "batch_internal.hpp"

namespace tplbm {
namespace {

constexpr int kNoallocMaxCols = 8192;
constexpr int kMaxDevices = 64;

// scratch layout: raw descriptions as the caller gave them, the kernel's
// descriptors (with node offsets), the processing order, the queue counter
constexpr size_t kRawBytes = sizeof(tplbm_column) * kNoallocMaxCols;
constexpr size_t kDescOff = (kRawBytes + 255) & ~(size_t)255;
constexpr size_t kDescBytes = sizeof(ColumnDesc) * kNoallocMaxCols;
constexpr size_t kOrderOff = kDescOff + ((kDescBytes + 255) & ~(size_t)255);
constexpr size_t kOrderBytes = sizeof(int) * kNoallocMaxCols;
constexpr size_t kQueueOff = kOrderOff + ((kOrderBytes + 255) & ~(size_t)255);
constexpr size_t kScratchBytes = kQueueOff + 256;

static_assert(sizeof(ColumnResult) == sizeof(tplbm_col_result) &&
                  offsetof(ColumnResult, steps) == offsetof(tplbm_col_result, steps) &&
                  offsetof(ColumnResult, status) == offsetof(tplbm_col_result, status) &&
                  offsetof(ColumnResult, mass) == offsetof(tplbm_col_result, mass) &&
                  offsetof(ColumnResult, max_u) == offsetof(tplbm_col_result, max_u),
              "the kernel writes tplbm_col_result records directly");

}  // namespace
}  // namespace tplbm

// The sweep's scratch on each GPU (about 480 KiB, held until the process ends).
static __device__ __align__(256) unsigned char scratch[tplbm::kScratchBytes];

namespace tplbm {
namespace {

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// Kernel descriptors from the caller's descriptions: node offsets are the
// exclusive prefix sum of the heights (each thread sums a contiguous chunk,
// then a block scan of the chunk sums); columns run in index order.  Also
// clears the queue counter of the launch that follows on the stream.
__global__ __launch_bounds__(1024) void batch_noalloc_prepare(const tplbm_column *raw, int ncols,
                                                              ColumnDesc *desc, int *order,
                                                              unsigned *queue)
{
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int per = (ncols + 1023) / 1024;
    const int k0 = t * per, k1 = min(k0 + per, ncols);
    long long s = 0;
    for (int k = k0; k < k1; ++k) s += raw[k].height;
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const long long v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long off = part[t] - s;
    for (int k = k0; k < k1; ++k) {
        const tplbm_column c = raw[k];
        ColumnDesc d;
        d.height = c.height;
        d.form = c.gravity_form;
        d.offset = off;
        d.g = c.g;
        d.rho_v = c.rho_v;
        desc[k] = d;
        order[k] = k;
        off += c.height;
    }
    if (t == 0) *queue = 0u;
}

}  // namespace
}  // namespace tplbm

using namespace tplbm;

extern "C" int tplbm_batch_run_noalloc(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                                       const double *dev_rho0, const double *dev_T0, double *dev_rho_out,
                                       double *dev_T_out, tplbm_col_result *dev_results, double tol,
                                       int64_t max_steps, int32_t check_every, void *hip_stream)
{
    int64_t total = 0;
    int rc = batch_validate(p, ncols, cols, &total);
    if (rc) return rc;
    if (ncols > kNoallocMaxCols)
        return batch_fail(TPLBM_ESHAPE, "%d columns: the allocation-free sweep takes at most %d", ncols,
                          kNoallocMaxCols);
    if (!dev_rho0 || !dev_T0 || !dev_rho_out || !dev_T_out || !dev_results)
        return batch_fail(TPLBM_EINVAL, "NULL device array");
    if (!(tol >= 0) || max_steps < 0 || check_every < 1)
        return batch_fail(TPLBM_EINVAL, "need tol >= 0, max_steps >= 0 and check_every >= 1");
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return batch_fail(TPLBM_EHIP, "scratch address: %s", hipGetErrorString(e));
    char *sc = (char *)base;
    tplbm_column *raw = (tplbm_column *)sc;
    ColumnDesc *desc = (ColumnDesc *)(sc + kDescOff);
    int *order = (int *)(sc + kOrderOff);
    unsigned *queue = (unsigned *)(sc + kQueueOff);
    hipStream_t s = (hipStream_t)hip_stream;
    e = hipMemcpyAsync(raw, cols, sizeof(tplbm_column) * ncols, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return batch_fail(TPLBM_EHIP, "copying the columns: %s", hipGetErrorString(e));
    hipLaunchKernelGGL(batch_noalloc_prepare, dim3(1), dim3(1024), 0, s, raw, ncols, desc, order, queue);
    e = hipGetLastError();
    if (e != hipSuccess) return batch_fail(TPLBM_EHIP, "preparing the columns: %s", hipGetErrorString(e));
    BatchArgs a;
    a.cols = desc;
    a.ncols = ncols;
    a.order = order;
    a.rho0 = dev_rho0;
    a.T0 = dev_T0;
    a.rho_out = dev_rho_out;
    a.T_out = dev_T_out;
    a.f_in = nullptr;
    a.f_out = nullptr;
    a.nodes = total;
    a.results = (ColumnResult *)dev_results;
    a.queue = queue;
    a.tol = tol;
    a.check_every = check_every;
    a.max_steps = max_steps;
    const int shape = 0;  // 256 threads x 8 nodes: holds every height up to 2048
    e = d1q3_batch_launch(shape, a, batch_phys(*p), batch_grid(shape, ncols), s);
    if (e != hipSuccess) return batch_fail(TPLBM_EHIP, "batch launch: %s", hipGetErrorString(e));
    // the columns were read from host memory that the caller may reuse at return
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return batch_fail(TPLBM_EHIP, "batch run: %s", hipGetErrorString(e));
    return TPLBM_OK;
}
