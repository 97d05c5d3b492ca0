// Host side of the batched column sweep (tplbm_batch_* in include/tplbm.h):
// workspace layout, longest-column-first ordering, the persistent launch and
// the autotuner that picks the kernel shape and the check interval.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tplbm.h"
#include "batch_internal.hpp"

using namespace tplbm;

struct tplbm_batch {
    tplbm_batch_params p;
    hipStream_t stream = nullptr;
    int ncols = 0;
    int64_t total = 0;
    std::vector<ColumnDesc> cols;
    std::vector<int> order;
    ColumnDesc *d_cols = nullptr;
    int *d_order = nullptr;
    int *d_sample = nullptr;  // autotuner trial order
    double *rho0 = nullptr, *T0 = nullptr, *rho_out = nullptr, *T_out = nullptr;
    double *f_end = nullptr;    // end-level populations of the last launch (3 planes)
    bool have_end = false;      // f_end/T_out hold the end of a tplbm_batch_run
    bool resume = false;        // the next run continues from f_end/T_out
    ColumnResult *results = nullptr;
    unsigned *queue = nullptr;
    int shape = 0, check_every = 100;
    int cus = 256;
    bool have_state = false;
    Phys phys;
    std::string err;
};

namespace {

thread_local std::string g_berr = "no error";

int bfail(tplbm_batch *b, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf; else g_berr = buf;
    return code;
}

#define BHIP(b, expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), TPLBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

constexpr int kMaxHeight = 2048;

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

int tplbm::batch_validate(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                          int64_t *total)
{
    if (!p || !cols || ncols <= 0) return bfail(nullptr, TPLBM_EINVAL, "need params, ncols > 0 and columns");
    if (p->eos != TPLBM_EOS_CARNAHAN_STARLING && p->eos != TPLBM_EOS_IDEAL_LATTICE)
        return bfail(nullptr, TPLBM_EINVAL, "unknown eos");
    if (p->eos == TPLBM_EOS_CARNAHAN_STARLING && !(p->G < 0 && p->a > 0 && p->b > 0 && p->R > 0))
        return bfail(nullptr, TPLBM_EINVAL, "C-S needs a, b, R > 0 and G < 0");
    if (!(p->cv > 0) || !(p->kappa >= 0)) return bfail(nullptr, TPLBM_EINVAL, "need c_v > 0, kappa >= 0");
    int64_t t = 0;
    for (int k = 0; k < ncols; ++k) {
        if (cols[k].height < 3 || cols[k].height > kMaxHeight)
            return bfail(nullptr, TPLBM_ESHAPE, "column %d: height %d outside 3..%d", k, cols[k].height, kMaxHeight);
        if (cols[k].gravity_form < 1 || cols[k].gravity_form > 3)
            return bfail(nullptr, TPLBM_EINVAL, "column %d: gravity_form must be 1, 2 or 3", k);
        if (!std::isfinite(cols[k].g)) return bfail(nullptr, TPLBM_EINVAL, "column %d: g not finite", k);
        if (!std::isfinite(cols[k].rho_v)) return bfail(nullptr, TPLBM_EINVAL, "column %d: rho_v not finite", k);
        t += cols[k].height;
    }
    *total = t;
    return TPLBM_OK;
}

int tplbm::batch_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_berr = buf;
    return code;
}

Phys tplbm::batch_phys(const tplbm_batch_params &p)
{
    Phys c;
    std::memset(&c, 0, sizeof c);
    c.a = p.a;
    c.b_quarter = p.b / 4.0;
    c.R = p.R;
    c.two_over_G = 2.0 / p.G;
    c.G = p.G;
    c.G2 = p.G * p.G;
    c.sigma = p.sigma;
    c.kappa_over_cv = p.kappa / p.cv;
    c.R_over_cv = p.R / p.cv;
    for (int k = 0; k < 9; ++k) c.lam[k] = 1.0;
    c.eos = p.eos;
    c.form = 1;
    return c;
}

int tplbm::batch_grid(int shape, int ncols)
{
    int per = 1, dev = 0, cus = 256;
    if (d1q3_batch_occupancy(shape, &per) != hipSuccess || per < 1) per = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return (int)std::min<long>((long)cus * per, ncols);
}

namespace {

struct BLayout {
    size_t cols, order, field, results, queue, total;
};

BLayout blayout(int ncols, int64_t total)
{
    BLayout L;
    L.cols = al(sizeof(ColumnDesc) * ncols);
    L.order = al(sizeof(int) * ncols);
    L.field = al(sizeof(double) * (size_t)total);
    L.results = al(sizeof(ColumnResult) * ncols);
    L.queue = 256;
    L.total = L.cols + 2 * L.order + 7 * L.field + L.results + L.queue;
    return L;
}

int grid_for(tplbm_batch *b, int shape)
{
    int per = 1;
    if (d1q3_batch_occupancy(shape, &per) != hipSuccess || per < 1) per = 1;
    long g = (long)b->cus * per;
    return (int)std::min<long>(g, b->ncols);
}

int run_once(tplbm_batch *b, const ColumnDesc *cols, const int *order, int ncols, int shape,
             int check_every, double tol, int64_t max_steps, float *ms, bool resume = false)
{
    BHIP(b, hipMemsetAsync(b->queue, 0, sizeof(unsigned), b->stream));
    BatchArgs a;
    a.cols = cols;
    a.ncols = ncols;
    a.order = order;
    a.rho0 = b->rho0;
    a.T0 = resume ? b->T_out : b->T0;
    a.rho_out = b->rho_out;
    a.T_out = b->T_out;
    a.f_in = resume ? b->f_end : nullptr;
    a.f_out = b->f_end;
    a.nodes = b->total;
    a.results = b->results;
    a.queue = b->queue;
    a.tol = tol;
    a.check_every = check_every;
    a.max_steps = max_steps;
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    BHIP(b, hipEventRecord(e0, b->stream));
    const int grid = std::min(grid_for(b, shape), ncols);
    hipError_t e = d1q3_batch_launch(shape, a, b->phys, grid, b->stream);
    if (e != hipSuccess) return bfail(b, TPLBM_EHIP, "batch launch: %s", hipGetErrorString(e));
    BHIP(b, hipEventRecord(e1, b->stream));
    BHIP(b, hipEventSynchronize(e1));
    float t = 0;
    BHIP(b, hipEventElapsedTime(&t, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (ms) *ms = t;
    return TPLBM_OK;
}

}  // namespace

extern "C" {

int tplbm_batch_workspace_bytes(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                                size_t *bytes)
{
    int64_t total;
    int rc = batch_validate(p, ncols, cols, &total);
    if (rc) return rc;
    if (!bytes) return bfail(nullptr, TPLBM_EINVAL, "bytes is NULL");
    *bytes = blayout(ncols, total).total;
    return TPLBM_OK;
}

int tplbm_batch_create(const tplbm_batch_params *p, int32_t ncols, const tplbm_column *cols,
                       void *dev_workspace, size_t bytes, void *hip_stream, tplbm_batch **out)
{
    int64_t total;
    int rc = batch_validate(p, ncols, cols, &total);
    if (rc) return rc;
    if (!out || !dev_workspace) return bfail(nullptr, TPLBM_EINVAL, "NULL argument");
    if (((uintptr_t)dev_workspace & 255) != 0) return bfail(nullptr, TPLBM_EINVAL, "workspace must be 256-byte aligned");
    const BLayout L = blayout(ncols, total);
    if (bytes < L.total) return bfail(nullptr, TPLBM_ESHAPE, "workspace has %zu bytes, need %zu", bytes, L.total);
    tplbm_batch *b = new tplbm_batch();
    b->p = *p;
    b->stream = (hipStream_t)hip_stream;
    b->ncols = ncols;
    b->total = total;
    b->cols.resize(ncols);
    int64_t off = 0;
    for (int k = 0; k < ncols; ++k) {
        b->cols[k].height = cols[k].height;
        b->cols[k].form = cols[k].gravity_form;
        b->cols[k].offset = off;
        b->cols[k].g = cols[k].g;
        b->cols[k].rho_v = cols[k].rho_v;
        off += cols[k].height;
    }
    // longest columns first: their time to steady state grows fastest with
    // height, so they start early and the short ones fill in at the end
    b->order.resize(ncols);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return b->cols[x].height > b->cols[y].height; });
    char *q = (char *)dev_workspace;
    b->d_cols = (ColumnDesc *)q; q += L.cols;
    b->d_order = (int *)q; q += L.order;
    b->d_sample = (int *)q; q += L.order;
    b->rho0 = (double *)q; q += L.field;
    b->T0 = (double *)q; q += L.field;
    b->rho_out = (double *)q; q += L.field;
    b->T_out = (double *)q; q += L.field;
    b->f_end = (double *)q; q += 3 * L.field;
    b->results = (ColumnResult *)q; q += L.results;
    b->queue = (unsigned *)q;
    b->phys = batch_phys(*p);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            b->cus = cus;
    }
    hipError_t e = hipMemcpyAsync(b->d_cols, b->cols.data(), sizeof(ColumnDesc) * ncols, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int) * ncols, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return bfail(nullptr, TPLBM_EHIP, "batch create: %s", hipGetErrorString(e));
    }
    *out = b;
    return TPLBM_OK;
}

int tplbm_batch_set_state(tplbm_batch *b, const double *rho, const double *T)
{
    if (!b || !rho || !T) return bfail(b, TPLBM_EINVAL, "NULL argument");
    BHIP(b, hipMemcpyAsync(b->rho0, rho, sizeof(double) * b->total, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->T0, T, sizeof(double) * b->total, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->have_state = true;
    b->have_end = false;
    b->resume = false;
    return TPLBM_OK;
}

int tplbm_batch_resume(tplbm_batch *b, const double *T_bot, const double *T_top)
{
    if (!b) return bfail(nullptr, TPLBM_EINVAL, "batch is NULL");
    if (!b->have_end) return bfail(b, TPLBM_EINVAL, "no run has ended since the last set_state or autotune");
    for (int k = 0; k < b->ncols; ++k) {
        if ((T_bot && !(T_bot[k] > 0 && std::isfinite(T_bot[k]))) ||
            (T_top && !(T_top[k] > 0 && std::isfinite(T_top[k]))))
            return bfail(b, TPLBM_EINVAL, "column %d: wall temperatures must be finite and > 0", k);
    }
    if (T_bot || T_top) {
        std::vector<double> T(b->total);
        BHIP(b, hipMemcpyAsync(T.data(), b->T_out, sizeof(double) * b->total, hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
        for (int k = 0; k < b->ncols; ++k) {
            const ColumnDesc &d = b->cols[k];
            if (T_bot) T[d.offset] = T_bot[k];
            if (T_top) T[d.offset + d.height - 1] = T_top[k];
        }
        BHIP(b, hipMemcpyAsync(b->T_out, T.data(), sizeof(double) * b->total, hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
    }
    b->resume = true;
    return TPLBM_OK;
}

int tplbm_batch_run(tplbm_batch *b, double tol, int64_t max_steps, tplbm_col_result *out)
{
    if (!b) return bfail(nullptr, TPLBM_EINVAL, "batch is NULL");
    if (!b->have_state) return bfail(b, TPLBM_EINVAL, "call tplbm_batch_set_state first");
    if (!(tol >= 0) || max_steps < 0) return bfail(b, TPLBM_EINVAL, "need tol >= 0 and max_steps >= 0");
    const bool resume = b->resume;
    b->resume = false;
    int rc = run_once(b, b->d_cols, b->d_order, b->ncols, b->shape, b->check_every, tol, max_steps, nullptr,
                      resume);
    if (rc) return rc;
    b->have_end = true;
    if (out) {
        std::vector<ColumnResult> r(b->ncols);
        BHIP(b, hipMemcpyAsync(r.data(), b->results, sizeof(ColumnResult) * b->ncols, hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));
        for (int k = 0; k < b->ncols; ++k) {
            out[k].steps = r[k].steps;
            out[k].status = r[k].status;
            out[k].pad = 0;
            out[k].mass = r[k].mass;
            out[k].max_u = r[k].max_u;
        }
    }
    return TPLBM_OK;
}

int tplbm_batch_read(tplbm_batch *b, int field, double *host_out)
{
    if (!b || !host_out) return bfail(b, TPLBM_EINVAL, "NULL argument");
    const double *src = field == TPLBM_RHO ? b->rho_out : field == TPLBM_T ? b->T_out : nullptr;
    if (!src) return bfail(b, TPLBM_EINVAL, "field must be TPLBM_RHO or TPLBM_T");
    BHIP(b, hipMemcpyAsync(host_out, src, sizeof(double) * b->total, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return TPLBM_OK;
}

int tplbm_batch_set_tuning(tplbm_batch *b, int32_t shape, int32_t check_every)
{
    if (!b) return bfail(nullptr, TPLBM_EINVAL, "batch is NULL");
    if (shape >= kNumBatchShapes || check_every < 0) return bfail(b, TPLBM_EINVAL, "bad tuning");
    if (shape >= 0) {
        int hmax = 0;
        for (auto &c : b->cols) hmax = std::max(hmax, (int)c.height);
        if (hmax > kBatchShapes[shape].threads * kBatchShapes[shape].nodes_per_thread)
            return bfail(b, TPLBM_ESHAPE, "shape %d holds at most %d nodes", shape,
                         kBatchShapes[shape].threads * kBatchShapes[shape].nodes_per_thread);
        b->shape = shape;
    }
    if (check_every > 0) b->check_every = check_every;
    return TPLBM_OK;
}

// The autotuner times every kernel shape that holds the tallest column on a
// trial sweep (a fixed number of steps for a sample of the batch, in the
// production order), keeps the fastest in node-steps per second, then picks
// the shortest check interval whose throughput stays within 3% of the best:
// a short interval stops converged columns sooner, a long one checks less.
int tplbm_batch_autotune(tplbm_batch *b, double budget_ms, tplbm_batch_tuning *out)
{
    if (!b) return bfail(nullptr, TPLBM_EINVAL, "batch is NULL");
    if (!b->have_state) return bfail(b, TPLBM_EINVAL, "call tplbm_batch_set_state first");
    // the trial launches overwrite the sampled columns' end state
    b->have_end = false;
    b->resume = false;
    int hmax = 0;
    for (auto &c : b->cols) hmax = std::max(hmax, (int)c.height);
    // trial sample: a stride through the production order, about two
    // resident waves of columns
    const int grid0 = grid_for(b, 0);
    const int nsample = std::min(b->ncols, std::max(1, 2 * grid0));
    std::vector<int> sample(nsample);
    for (int k = 0; k < nsample; ++k) sample[k] = b->order[(size_t)k * b->ncols / nsample];
    int64_t sample_nodes = 0;
    for (int k : sample) sample_nodes += b->cols[k].height;
    int *d_sample = b->d_sample;
    BHIP(b, hipMemcpyAsync(d_sample, sample.data(), sizeof(int) * nsample, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    const int64_t trial_steps = 400;
    double spent = 0.0, best = -1.0;
    int best_shape = b->shape;
    for (int s = 0; s < kNumBatchShapes; ++s) {
        if (hmax > kBatchShapes[s].threads * kBatchShapes[s].nodes_per_thread) continue;
        float ms = 0;
        // tol = 0: no column stops early, every column runs trial_steps
        int rc = run_once(b, b->d_cols, d_sample, nsample, s, 1 << 30, 0.0, trial_steps, &ms);
        if (rc) return rc;
        spent += ms;
        const double rate = (double)sample_nodes * trial_steps / (ms * 1e-3);
        if (rate > best) { best = rate; best_shape = s; }
        if (spent > budget_ms) break;
    }
    const int Ks[] = {25, 50, 100, 200, 400};
    double rates[5];
    double kbest = 0.0;
    for (int i = 0; i < 5; ++i) {
        float ms = 0;
        int rc = run_once(b, b->d_cols, d_sample, nsample, best_shape, Ks[i], 0.0, trial_steps, &ms);
        if (rc) return rc;
        rates[i] = (double)sample_nodes * trial_steps / (ms * 1e-3);
        kbest = std::max(kbest, rates[i]);
    }
    int K = Ks[4];
    for (int i = 0; i < 5; ++i)
        if (rates[i] >= 0.97 * kbest) { K = Ks[i]; break; }
    b->shape = best_shape;
    b->check_every = K;
    if (out) {
        out->shape = best_shape;
        out->threads = kBatchShapes[best_shape].threads;
        out->nodes_per_thread = kBatchShapes[best_shape].nodes_per_thread;
        out->check_every = K;
        out->grid = grid_for(b, best_shape);
        out->pad = 0;
        out->node_steps_per_s = best;
    }
    return TPLBM_OK;
}

void tplbm_batch_destroy(tplbm_batch *b) { delete b; }

const char *tplbm_batch_last_error(const tplbm_batch *b) { return b ? b->err.c_str() : g_berr.c_str(); }

}  // extern "C"
