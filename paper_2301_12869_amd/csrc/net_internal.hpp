// Internal interface between the warm-start network's host code and kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tplbm {

// layer shapes: 8 -> 64 -> 64 -> 64 -> 64 -> 64 -> 2, width-5 taps
constexpr int kNetLayers = 6;
constexpr int kNetTaps = 5;
constexpr int kNetCin[kNetLayers] = {8, 64, 64, 64, 64, 64};
constexpr int kNetCout[kNetLayers] = {64, 64, 64, 64, 64, 2};
constexpr int kNetCoutPad[kNetLayers] = {64, 64, 64, 64, 64, 32};  // forward GEMM rows
constexpr int kNetGradCin[kNetLayers] = {0, 64, 64, 64, 64, 8};    // dZ channels read by dX

struct NetCol {
    int32_t height;     // nodes including both wall nodes
    int32_t form;       // gravity form 1 or 2
    double t_reduced;   // T / T_c
    double g;           // gravity magnitude
    double mean_reduced;  // <rho> / rho_c
    double lever_height;  // lever-rule interface height (nodes)
    int64_t offset;     // first node in the dataset arrays (training columns)
};

struct NetEntry {
    int32_t src;        // index into the column table
    int32_t pad;
    int64_t pos;        // first position of the column in the padded layout
    int64_t out;        // first node of the column in concatenated outputs
};

hipError_t net_prep(const NetCol *cols, const NetEntry *entries, int n, const double *rho, const double *T,
                    double rho_c, double T_c, uint16_t *x, uint8_t *guard, float *tgt, hipStream_t s);
hipError_t net_emit(const NetCol *cols, const NetEntry *entries, int n, const float *out, double rho_c,
                    double T_c, double *rho_out, double *T_out, hipStream_t s);
hipError_t net_raw_out(const NetCol *cols, const NetEntry *entries, int n, const float *out, float *dst,
                       hipStream_t s);
hipError_t net_conv_forward(int layer, const uint16_t *in, const uint16_t *W, const float *bias, int64_t P,
                            const uint8_t *guard, uint16_t *out_bf16, float *out_f32, hipStream_t s);
// one ordered reduction dst[e] = sum_b src[b * stride + e], e < n, b < nb
struct RedJob {
    const float *src;
    int nb, stride, n;
    float *dst;
};
// input gradient of layer `layer` (masked by its input act_in) in BF16, and
// per-block channel sums of it (the bias gradient of layer - 1) into bsum:
// *nbsum rows of 64 floats (at most 512)
hipError_t net_conv_input_grad(int layer, const uint16_t *dZ, const uint16_t *Wg, int64_t P, const uint8_t *guard,
                               const uint16_t *act_in, uint16_t *dprev_bf16, float *bsum, int *nbsum, hipStream_t s);
// weight gradient of a layer, reduced together with its bias gradient
// (`bias`, the partials of net_conv_input_grad or net_bias_partials)
hipError_t net_weight_grad(int layer, const uint16_t *dZ, const uint16_t *X, int64_t P, int nblocks,
                           float *partial, float *dW, const RedJob &bias, hipStream_t s);
// per-slice channel sums of an FP32 dZ with zs channels per position
// (*nparts rows of zs floats)
hipError_t net_bias_partials(int zs, const float *dZ, int64_t P, int nblocks, float *partial, int *nparts,
                             hipStream_t s);
hipError_t net_loss(const float *out, const float *tgt, const uint8_t *guard, int64_t P, float scale, float *dZf,
                    uint16_t *dZb, float *partial, int nblocks, hipStream_t s);
hipError_t net_adam(float *theta, const float *grad, float *m, float *v, int n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s);
// the FP32 weights of every layer and their BF16 copies (Wg[0] unused)
struct NetWeightSet {
    const float *Wf[kNetLayers];
    uint16_t *Wb[kNetLayers];
    uint16_t *Wg[kNetLayers];
};
hipError_t net_prep_weights(const NetWeightSet &w, hipStream_t s);
hipError_t net_mfma_probe(const uint16_t *a, const uint16_t *b, float *d, hipStream_t s);

}  // namespace tplbm
