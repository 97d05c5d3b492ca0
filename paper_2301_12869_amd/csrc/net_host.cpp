// Host side of the warm-start network (tplbm_net_* in include/tplbm.h):
// workspace layout, the padded position layout of a batch of columns, and
// the forward / backward / Adam sequence of kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tplbm.h"
#include "net_internal.hpp"

using namespace tplbm;

namespace {

constexpr int kMaxHeight = 2048;
constexpr int kSlices = 256;        // position slices of the weight-gradient reduction
constexpr int kLossBlocks = 256;
constexpr int kPartialStride = 64 * 5 * 64;
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t param_count()
{
    int64_t n = 0;
    for (int l = 0; l < kNetLayers; ++l) n += (int64_t)kNetCout[l] * kNetTaps * kNetCin[l] + kNetCout[l];
    return n;
}

int64_t w_offset(int layer)
{
    int64_t n = 0;
    for (int l = 0; l < layer; ++l) n += (int64_t)kNetCout[l] * kNetTaps * kNetCin[l] + kNetCout[l];
    return n;
}

int64_t b_offset(int layer) { return w_offset(layer) + (int64_t)kNetCout[layer] * kNetTaps * kNetCin[layer]; }

struct NLayout {
    size_t theta, wb[kNetLayers], wg[kNetLayers], dcols, dfield, cols, entries;
    size_t x, act, out2, guard, dz8f, dz8b, dab, partial, bpart, loss, pred, raw;
    size_t total;
    int64_t P;
};

NLayout nlayout(const tplbm_net_config &c)
{
    NLayout L{};
    const int64_t np = param_count();
    L.P = c.max_nodes + 2 * (int64_t)c.max_cols + 2;
    const size_t P = (size_t)L.P;
    L.theta = al(sizeof(float) * np);
    for (int l = 0; l < kNetLayers; ++l) {
        L.wb[l] = al(2 * (size_t)kNetCoutPad[l] * kNetTaps * kNetCin[l]);
        L.wg[l] = l ? al(2 * (size_t)kNetCin[l] * kNetTaps * kNetGradCin[l]) : 0;
    }
    L.dcols = al(sizeof(NetCol) * (size_t)c.dataset_cols);
    L.dfield = al(sizeof(double) * (size_t)c.dataset_nodes);
    L.cols = al(sizeof(NetCol) * (size_t)c.max_cols);
    L.entries = al(sizeof(NetEntry) * (size_t)c.max_cols);
    L.x = al(2 * 8 * P);
    L.act = al(2 * 64 * P);
    L.out2 = al(4 * 2 * P);
    L.guard = al(P);
    L.dz8f = al(4 * 8 * P);
    L.dz8b = al(2 * 8 * P);
    L.dab = al(2 * 64 * P);
    L.partial = al(sizeof(float) * (size_t)kSlices * kPartialStride);
    // bias-gradient partials: at most 512 convolution blocks x 64 channels,
    // or kSlices x 8 for the output layer
    L.bpart = al(sizeof(float) * (size_t)(512 * 64 > kSlices * 8 ? 512 * 64 : kSlices * 8));
    L.loss = al(sizeof(float) * kLossBlocks);
    L.pred = al(sizeof(double) * (size_t)c.max_nodes);
    L.raw = al(sizeof(float) * 2 * (size_t)c.max_nodes);
    size_t t = 4 * L.theta;
    for (int l = 0; l < kNetLayers; ++l) t += L.wb[l] + L.wg[l];
    t += L.dcols + 2 * L.dfield + L.cols + L.entries + L.x + 5 * L.act + 2 * L.out2 + L.guard + L.dz8f + L.dz8b +
         2 * L.dab + L.partial + L.bpart + L.loss + 2 * L.pred + L.raw;
    L.total = t;
    return L;
}

thread_local std::string g_nerr = "no error";

}  // namespace

struct tplbm_net {
    tplbm_net_config c;
    hipStream_t stream = nullptr;
    int64_t np = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wb[kNetLayers] = {}, *wg[kNetLayers] = {};
    NetCol *dcols = nullptr, *cols = nullptr;
    double *drho = nullptr, *dT = nullptr;
    NetEntry *entries = nullptr;
    uint16_t *x = nullptr, *act[kNetLayers] = {};  // act[0] = x
    float *out = nullptr, *tgt = nullptr;
    uint8_t *guard = nullptr;
    float *dz8f = nullptr;
    uint16_t *dz8b = nullptr, *dab[2] = {};
    float *partial = nullptr, *bpart = nullptr, *loss = nullptr;
    double *pred_rho = nullptr, *pred_T = nullptr;
    float *raw = nullptr;
    std::vector<tplbm_net_column> data;  // host copy of the training columns
    std::vector<int64_t> data_off;
    int data_cols = 0;
    int64_t adam_t = 0;
    bool have_params = false;
    std::string err;
};

namespace {

int nfail(tplbm_net *n, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n) n->err = buf; else g_nerr = buf;
    return code;
}

#define NHIP(n, expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return nfail((n), TPLBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

int check_column(tplbm_net *n, const tplbm_net_column &c, int k)
{
    if (c.height < 3 || c.height > kMaxHeight)
        return nfail(n, TPLBM_ESHAPE, "column %d: height %d outside 3..%d", k, c.height, kMaxHeight);
    if (c.gravity_form != 1 && c.gravity_form != 2)
        return nfail(n, TPLBM_EINVAL, "column %d: gravity_form must be 1 or 2", k);
    if (!(c.g > 0) || !std::isfinite(c.g) || !std::isfinite(c.t_reduced) || !std::isfinite(c.mean_reduced) ||
        !std::isfinite(c.lever_height))
        return nfail(n, TPLBM_EINVAL, "column %d: need finite t_reduced, mean_reduced, lever_height and g > 0", k);
    return TPLBM_OK;
}

NetCol to_dev(const tplbm_net_column &c, int64_t offset)
{
    NetCol d;
    d.height = c.height;
    d.form = c.gravity_form;
    d.t_reduced = c.t_reduced;
    d.g = c.g;
    d.mean_reduced = c.mean_reduced;
    d.lever_height = c.lever_height;
    d.offset = offset;
    return d;
}

// Entries for columns with the given heights; returns the number of positions.
int64_t make_entries(const std::vector<int> &src, const std::vector<int> &heights, std::vector<NetEntry> &e)
{
    e.resize(src.size());
    int64_t pos = 2, out = 0;
    for (size_t k = 0; k < src.size(); ++k) {
        e[k].src = src[k];
        e[k].pad = 0;
        e[k].pos = pos;
        e[k].out = out;
        pos += heights[k] + 2;
        out += heights[k];
    }
    return pos;
}

int upload_entries(tplbm_net *n, const std::vector<NetEntry> &e)
{
    NHIP(n, hipMemcpyAsync(n->entries, e.data(), sizeof(NetEntry) * e.size(), hipMemcpyHostToDevice, n->stream));
    return TPLBM_OK;
}

int forward(tplbm_net *n, int64_t P)
{
    for (int l = 0; l < kNetLayers; ++l) {
        const float *bias = n->theta + b_offset(l);
        if (l < kNetLayers - 1)
            NHIP(n, net_conv_forward(l, n->act[l], n->wb[l], bias, P, n->guard, n->act[l + 1], nullptr, n->stream));
        else
            NHIP(n, net_conv_forward(l, n->act[l], n->wb[l], bias, P, n->guard, nullptr, n->out, n->stream));
    }
    return TPLBM_OK;
}

// loss and gradient (into n->grad) of the columns whose entries were uploaded
int loss_and_grad(tplbm_net *n, int64_t P, int64_t nodes, double *loss)
{
    int rc = forward(n, P);
    if (rc) return rc;
    const float scale = (float)(1.0 / (2.0 * (double)nodes));
    NHIP(n, net_loss(n->out, n->tgt, n->guard, P, scale, n->dz8f, n->dz8b, n->loss, kLossBlocks, n->stream));
    // layer 5: dZ has 8 channels (2 real)
    const uint16_t *dzb = n->dz8b;
    const float *dzf = n->dz8f;
    int cur = 0;
    // each layer's bias partials come from the output layer's FP32 dZ or
    // from the input gradient that produced its dZ, and are reduced in the
    // launch that reduces its weight gradient
    int nbias = 0, bstride = 8;
    NHIP(n, net_bias_partials(8, dzf, P, kSlices, n->bpart, &nbias, n->stream));
    for (int l = kNetLayers - 1; l >= 0; --l) {
        const RedJob bias{n->bpart, nbias, bstride, kNetCout[l], n->grad + b_offset(l)};
        NHIP(n, net_weight_grad(l, dzb, n->act[l], P, kSlices, n->partial, n->grad + w_offset(l), bias, n->stream));
        if (l == 0) break;
        NHIP(n, net_conv_input_grad(l, dzb, n->wg[l], P, n->guard, n->act[l], n->dab[cur], n->bpart, &nbias,
                                    n->stream));
        bstride = 64;
        dzb = n->dab[cur];
        cur ^= 1;
    }
    if (loss) {
        float part[kLossBlocks];
        NHIP(n, hipMemcpyAsync(part, n->loss, sizeof part, hipMemcpyDeviceToHost, n->stream));
        NHIP(n, hipStreamSynchronize(n->stream));
        double s = 0.0;
        for (int b = 0; b < kLossBlocks; ++b) s += part[b];
        *loss = s / (2.0 * (double)nodes);
    }
    return TPLBM_OK;
}

int prep_weights(tplbm_net *n)
{
    NetWeightSet w;
    for (int l = 0; l < kNetLayers; ++l) {
        w.Wf[l] = n->theta + w_offset(l);
        w.Wb[l] = n->wb[l];
        w.Wg[l] = l ? n->wg[l] : nullptr;
    }
    NHIP(n, net_prep_weights(w, n->stream));
    return TPLBM_OK;
}

// entries for a minibatch of dataset columns; returns positions and nodes
int dataset_batch(tplbm_net *n, int32_t nbatch, const int32_t *idx, int64_t *P, int64_t *nodes)
{
    if (!n->data_cols) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_dataset first");
    if (!idx || nbatch <= 0 || nbatch > n->c.max_cols)
        return nfail(n, TPLBM_EINVAL, "need 1..%d column indices", n->c.max_cols);
    std::vector<int> src(nbatch), h(nbatch);
    int64_t tot = 0;
    for (int k = 0; k < nbatch; ++k) {
        if (idx[k] < 0 || idx[k] >= n->data_cols)
            return nfail(n, TPLBM_EINVAL, "index %d outside the dataset (%d columns)", idx[k], n->data_cols);
        src[k] = idx[k];
        h[k] = n->data[idx[k]].height;
        tot += h[k];
    }
    if (tot > n->c.max_nodes) return nfail(n, TPLBM_ESHAPE, "batch has %lld nodes, max_nodes is %lld",
                                           (long long)tot, (long long)n->c.max_nodes);
    std::vector<NetEntry> e;
    *P = make_entries(src, h, e);
    *nodes = tot;
    int rc = upload_entries(n, e);
    if (rc) return rc;
    NHIP(n, net_prep(n->dcols, n->entries, nbatch, n->drho, n->dT, n->c.rho_c, n->c.T_c, n->x, n->guard, n->tgt,
                     n->stream));
    return TPLBM_OK;
}

// entries for caller columns (staged into n->cols); returns positions and nodes
int direct_batch(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, int64_t *P, int64_t *nodes)
{
    if (!cols || ncols <= 0 || ncols > n->c.max_cols)
        return nfail(n, TPLBM_EINVAL, "need 1..%d columns", n->c.max_cols);
    std::vector<NetCol> dc(ncols);
    std::vector<int> src(ncols), h(ncols);
    int64_t tot = 0;
    for (int k = 0; k < ncols; ++k) {
        int rc = check_column(n, cols[k], k);
        if (rc) return rc;
        dc[k] = to_dev(cols[k], 0);
        src[k] = k;
        h[k] = cols[k].height;
        tot += h[k];
    }
    if (tot > n->c.max_nodes) return nfail(n, TPLBM_ESHAPE, "columns have %lld nodes, max_nodes is %lld",
                                           (long long)tot, (long long)n->c.max_nodes);
    NHIP(n, hipMemcpyAsync(n->cols, dc.data(), sizeof(NetCol) * ncols, hipMemcpyHostToDevice, n->stream));
    std::vector<NetEntry> e;
    *P = make_entries(src, h, e);
    *nodes = tot;
    int rc = upload_entries(n, e);
    if (rc) return rc;
    NHIP(n, net_prep(n->cols, n->entries, ncols, nullptr, nullptr, n->c.rho_c, n->c.T_c, n->x, n->guard, nullptr,
                     n->stream));
    return TPLBM_OK;
}

int validate_config(const tplbm_net_config *c)
{
    if (!c) return nfail(nullptr, TPLBM_EINVAL, "config is NULL");
    if (!(c->rho_c > 0) || !(c->T_c > 0)) return nfail(nullptr, TPLBM_EINVAL, "need rho_c > 0 and T_c > 0");
    if (c->max_cols < 1 || c->max_nodes < 3) return nfail(nullptr, TPLBM_EINVAL, "need max_cols >= 1, max_nodes >= 3");
    if (c->dataset_cols < 0 || c->dataset_nodes < 0) return nfail(nullptr, TPLBM_EINVAL, "negative dataset size");
    // positions times 64 channels must stay within 32-bit element indices
    if (c->max_nodes + 2 * (int64_t)c->max_cols + 2 > (int64_t(1) << 25))
        return nfail(nullptr, TPLBM_ESHAPE, "at most 2^25 positions per call");
    return TPLBM_OK;
}

}  // namespace

extern "C" {

int tplbm_net_num_params(int64_t *n)
{
    if (!n) return nfail(nullptr, TPLBM_EINVAL, "NULL argument");
    *n = param_count();
    return TPLBM_OK;
}

int tplbm_net_workspace_bytes(const tplbm_net_config *c, size_t *bytes)
{
    int rc = validate_config(c);
    if (rc) return rc;
    if (!bytes) return nfail(nullptr, TPLBM_EINVAL, "bytes is NULL");
    *bytes = nlayout(*c).total;
    return TPLBM_OK;
}

int tplbm_net_create(const tplbm_net_config *c, void *dev_workspace, size_t bytes, void *hip_stream,
                     tplbm_net **out)
{
    int rc = validate_config(c);
    if (rc) return rc;
    if (!out || !dev_workspace) return nfail(nullptr, TPLBM_EINVAL, "NULL argument");
    if (((uintptr_t)dev_workspace & 255) != 0) return nfail(nullptr, TPLBM_EINVAL, "workspace must be 256-byte aligned");
    const NLayout L = nlayout(*c);
    if (bytes < L.total) return nfail(nullptr, TPLBM_ESHAPE, "workspace has %zu bytes, need %zu", bytes, L.total);
    tplbm_net *n = new tplbm_net();
    n->c = *c;
    n->stream = (hipStream_t)hip_stream;
    n->np = param_count();
    char *q = (char *)dev_workspace;
    n->theta = (float *)q; q += L.theta;
    n->grad = (float *)q; q += L.theta;
    n->m = (float *)q; q += L.theta;
    n->v = (float *)q; q += L.theta;
    for (int l = 0; l < kNetLayers; ++l) {
        n->wb[l] = (uint16_t *)q; q += L.wb[l];
        if (l) { n->wg[l] = (uint16_t *)q; q += L.wg[l]; }
    }
    n->dcols = (NetCol *)q; q += L.dcols;
    n->drho = (double *)q; q += L.dfield;
    n->dT = (double *)q; q += L.dfield;
    n->cols = (NetCol *)q; q += L.cols;
    n->entries = (NetEntry *)q; q += L.entries;
    n->x = (uint16_t *)q; q += L.x;
    n->act[0] = n->x;
    for (int l = 1; l < kNetLayers; ++l) { n->act[l] = (uint16_t *)q; q += L.act; }
    n->out = (float *)q; q += L.out2;
    n->tgt = (float *)q; q += L.out2;
    n->guard = (uint8_t *)q; q += L.guard;
    n->dz8f = (float *)q; q += L.dz8f;
    n->dz8b = (uint16_t *)q; q += L.dz8b;
    for (int k = 0; k < 2; ++k) { n->dab[k] = (uint16_t *)q; q += L.dab; }
    n->partial = (float *)q; q += L.partial;
    n->bpart = (float *)q; q += L.bpart;
    n->loss = (float *)q; q += L.loss;
    n->pred_rho = (double *)q; q += L.pred;
    n->pred_T = (double *)q; q += L.pred;
    n->raw = (float *)q;
    *out = n;
    return TPLBM_OK;
}

int tplbm_net_set_params(tplbm_net *n, const float *theta)
{
    if (!n || !theta) return nfail(n, TPLBM_EINVAL, "NULL argument");
    for (int64_t k = 0; k < n->np; ++k)
        if (!std::isfinite(theta[k])) return nfail(n, TPLBM_EINVAL, "parameter %lld is not finite", (long long)k);
    NHIP(n, hipMemcpyAsync(n->theta, theta, sizeof(float) * n->np, hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipMemsetAsync(n->m, 0, sizeof(float) * n->np, n->stream));
    NHIP(n, hipMemsetAsync(n->v, 0, sizeof(float) * n->np, n->stream));
    int rc = prep_weights(n);
    if (rc) return rc;
    NHIP(n, hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    n->have_params = true;
    return TPLBM_OK;
}

int tplbm_net_init(tplbm_net *n, uint64_t seed)
{
    if (!n) return nfail(nullptr, TPLBM_EINVAL, "net is NULL");
    // He-uniform weights, bound sqrt(6 / fan_in) with fan_in = 5 C_in, zero
    // biases.  Draw k (counted over the weights of every layer in order) is
    // the SplitMix64 finaliser of seed + (k + 1) * 0x9E3779B97F4A7C15 (Steele,
    // Lea and Flood, OOPSLA 2014), mapped to [-1, 1) from its top 53 bits.
    std::vector<float> theta(n->np, 0.0f);
    uint64_t k = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        const double bound = std::sqrt(6.0 / (double)(kNetTaps * kNetCin[l]));
        const int64_t nw = (int64_t)kNetCout[l] * kNetTaps * kNetCin[l], off = w_offset(l);
        for (int64_t e = 0; e < nw; ++e, ++k) {
            uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            const double u = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
            theta[off + e] = (float)(bound * u);
        }
    }
    return tplbm_net_set_params(n, theta.data());
}

int tplbm_net_get_params(tplbm_net *n, float *theta)
{
    if (!n || !theta) return nfail(n, TPLBM_EINVAL, "NULL argument");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    NHIP(n, hipMemcpyAsync(theta, n->theta, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

int tplbm_net_set_dataset(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, const double *rho,
                          const double *T)
{
    if (!n || !cols || !rho || !T || ncols <= 0) return nfail(n, TPLBM_EINVAL, "NULL argument or no columns");
    if (ncols > n->c.dataset_cols)
        return nfail(n, TPLBM_ESHAPE, "%d columns, the workspace holds %d", ncols, n->c.dataset_cols);
    std::vector<NetCol> dc(ncols);
    std::vector<int64_t> off(ncols);
    int64_t tot = 0;
    for (int k = 0; k < ncols; ++k) {
        int rc = check_column(n, cols[k], k);
        if (rc) return rc;
        off[k] = tot;
        dc[k] = to_dev(cols[k], tot);
        tot += cols[k].height;
    }
    if (tot > n->c.dataset_nodes)
        return nfail(n, TPLBM_ESHAPE, "%lld nodes, the workspace holds %lld", (long long)tot,
                     (long long)n->c.dataset_nodes);
    NHIP(n, hipMemcpyAsync(n->dcols, dc.data(), sizeof(NetCol) * ncols, hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipMemcpyAsync(n->drho, rho, sizeof(double) * tot, hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipMemcpyAsync(n->dT, T, sizeof(double) * tot, hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    n->data.assign(cols, cols + ncols);
    n->data_off = off;
    n->data_cols = ncols;
    return TPLBM_OK;
}

int tplbm_net_loss_grad(tplbm_net *n, int32_t nbatch, const int32_t *idx, double *loss, float *grad)
{
    if (!n) return nfail(nullptr, TPLBM_EINVAL, "net is NULL");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    int64_t P, nodes;
    int rc = dataset_batch(n, nbatch, idx, &P, &nodes);
    if (rc) return rc;
    rc = loss_and_grad(n, P, nodes, loss);
    if (rc) return rc;
    if (grad) NHIP(n, hipMemcpyAsync(grad, n->grad, sizeof(float) * n->np, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

int tplbm_net_train_step(tplbm_net *n, int32_t nbatch, const int32_t *idx, float lr, double *loss)
{
    if (!n) return nfail(nullptr, TPLBM_EINVAL, "net is NULL");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    if (!(lr > 0) || !std::isfinite(lr)) return nfail(n, TPLBM_EINVAL, "need a finite lr > 0");
    int64_t P, nodes;
    int rc = dataset_batch(n, nbatch, idx, &P, &nodes);
    if (rc) return rc;
    rc = loss_and_grad(n, P, nodes, loss);
    if (rc) return rc;
    n->adam_t += 1;
    // bias corrections from the FP32 betas the kernel uses, so that a constant
    // gradient gives corrected moments of exactly g and g^2 up to rounding
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)kBeta1, (double)n->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)kBeta2, (double)n->adam_t)));
    NHIP(n, net_adam(n->theta, n->grad, n->m, n->v, (int)n->np, lr, kBeta1, kBeta2, kEps, c1, c2, n->stream));
    rc = prep_weights(n);
    if (rc) return rc;
    if (!loss) NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

int tplbm_net_forward(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, float *out)
{
    if (!n || !out) return nfail(n, TPLBM_EINVAL, "NULL argument");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    int64_t P, nodes;
    int rc = direct_batch(n, ncols, cols, &P, &nodes);
    if (rc) return rc;
    rc = forward(n, P);
    if (rc) return rc;
    NHIP(n, net_raw_out(n->cols, n->entries, ncols, n->out, n->raw, n->stream));
    NHIP(n, hipMemcpyAsync(out, n->raw, sizeof(float) * 2 * nodes, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

int tplbm_net_predict(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, double *rho, double *T)
{
    if (!n || !rho || !T) return nfail(n, TPLBM_EINVAL, "NULL argument");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    int64_t P, nodes;
    int rc = direct_batch(n, ncols, cols, &P, &nodes);
    if (rc) return rc;
    rc = forward(n, P);
    if (rc) return rc;
    NHIP(n, net_emit(n->cols, n->entries, ncols, n->out, n->c.rho_c, n->c.T_c, n->pred_rho, n->pred_T, n->stream));
    NHIP(n, hipMemcpyAsync(rho, n->pred_rho, sizeof(double) * nodes, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipMemcpyAsync(T, n->pred_T, sizeof(double) * nodes, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

int tplbm_net_predict_device(tplbm_net *n, int32_t ncols, const tplbm_net_column *cols, double *dev_rho,
                             double *dev_T)
{
    if (!n || !dev_rho || !dev_T) return nfail(n, TPLBM_EINVAL, "NULL argument");
    if (!n->have_params) return nfail(n, TPLBM_EINVAL, "call tplbm_net_set_params first");
    int64_t P, nodes;
    int rc = direct_batch(n, ncols, cols, &P, &nodes);
    if (rc) return rc;
    rc = forward(n, P);
    if (rc) return rc;
    NHIP(n, net_emit(n->cols, n->entries, ncols, n->out, n->c.rho_c, n->c.T_c, n->pred_rho, n->pred_T, n->stream));
    NHIP(n, hipMemcpyAsync(dev_rho, n->pred_rho, sizeof(double) * nodes, hipMemcpyDeviceToDevice, n->stream));
    NHIP(n, hipMemcpyAsync(dev_T, n->pred_T, sizeof(double) * nodes, hipMemcpyDeviceToDevice, n->stream));
    return TPLBM_OK;
}

int tplbm_net_mfma_check(tplbm_net *n, const uint16_t *a, const uint16_t *b, float *d)
{
    if (!n || !a || !b || !d) return nfail(n, TPLBM_EINVAL, "NULL argument");
    // operands and result are staged in the partial-sum area (free between calls)
    uint16_t *da = (uint16_t *)n->partial;
    uint16_t *db = da + 512;
    float *dd = (float *)(db + 512);
    NHIP(n, hipMemcpyAsync(da, a, 2 * 512, hipMemcpyHostToDevice, n->stream));
    NHIP(n, hipMemcpyAsync(db, b, 2 * 512, hipMemcpyHostToDevice, n->stream));
    NHIP(n, net_mfma_probe(da, db, dd, n->stream));
    NHIP(n, hipMemcpyAsync(d, dd, sizeof(float) * 1024, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return TPLBM_OK;
}

void tplbm_net_destroy(tplbm_net *n) { delete n; }

const char *tplbm_net_last_error(const tplbm_net *n) { return n ? n->err.c_str() : g_nerr.c_str(); }

}  // extern "C"
