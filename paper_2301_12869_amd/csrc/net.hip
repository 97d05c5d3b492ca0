// Warm-start network kernels for gfx950: 1-D convolutions as implicit GEMMs
// on the BF16 matrix cores (gfx950's v_mfma_f32_32x32x16_bf16, FP32
// accumulation: K = 16 per instruction, lanes 0..31 and 32..63 each holding
// eight consecutive k of their row or column).
//
// A batch of columns is laid out position-major, channels fastest, with two
// all-zero guard positions between columns (and at both ends): a width-5
// convolution then never mixes columns, and its zero padding is exact
// without per-tap masks.  Outputs and gradients at guard positions are
// forced to zero, so every kernel writes every position it owns.
//
// Kernels:
//   conv_mfma   out[p][o] = sum_{t,i} W[o][t][i] in[p + t - 2][i]  (+ bias
//               and ReLU, or a mask by the layer input) -- forward layers
//               and, with flipped transposed weights, the input gradient,
//               whose per-block channel sums give the previous layer's bias
//               gradient
//   dw_mfma     partial dW[o][t][i] = sum_p dZ[p][o] X[p + t - 2][i] over a
//               slice of positions (operands staged transposed in LDS),
//               reduced in a fixed order afterwards (deterministic)
//   prep / emit / loss / adam / weight conversion in FP32 or FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "net_internal.hpp"

namespace tplbm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ __bf16 as_bf(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Accumulator element r of a lane holds D[row][col] of the 32 x 32 tile with
// col = lane % 32 and row = 8 (r / 4) + 4 (lane / 32) + r % 4.
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// MODE 0: hidden forward layer: out_bf16 = bf16(relu(acc + bias))
// MODE 1: output layer:         out_f32[p][o] = acc + bias for o < NOUT
// MODE 2: input gradient:       g = acc * (mask[p][o] > 0); out_bf16 = bf16(g), and the
//                               block's sums of g over its positions per channel (the
//                               previous layer's bias gradient) into bsum[block][o]
// Persistent blocks of 4 waves: the layer's BF16 weights are staged in LDS
// once per block (rows padded by 8 elements: 16-byte rows for the 8-element
// fragments), then the block walks 128-position tiles; each wave owns 32
// positions and all 32 NTILES output channels, so one activation fragment
// feeds NTILES MFMAs.  K runs over (tap, input channel), 16 at a time; with
// 8 input channels the last step's upper half (a sixth tap) is zero.  A
// tile's 132 input positions (2 on each side for the taps) are staged in LDS
// too, read with 16-byte loads one tile ahead, so each activation is read
// from memory once per tile rather than once per tap.
template <int CIN, int NTILES, int MODE, int NOUT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void conv_mfma(const uint16_t *__restrict__ in, const uint16_t *__restrict__ W,
                                                 const float *__restrict__ bias, int P,
                                                 const uint8_t *__restrict__ guard,
                                                 const uint16_t *__restrict__ mask, float *__restrict__ out_f32,
                                                 uint16_t *__restrict__ out_bf16, float *__restrict__ bsum)
{
    constexpr int COUT = 32 * NTILES;
    constexpr int ROW = 5 * CIN;       // weights of one output channel
    constexpr int RS = ROW + 8;        // padded LDS row
    constexpr int KS = (ROW + 15) / 16;  // K steps
    constexpr int NTHR = 64 * WAVES;   // threads of a block
    constexpr int TPOS = 32 * WAVES;   // positions of a tile (32 a wave)
    constexpr int TP = TPOS + 4;       // staged positions of a tile
    constexpr int AS = CIN + 8;        // padded LDS row of a staged position
    constexpr int AV = CIN / 8;        // 16-byte groups of a position
    constexpr int NA = (TP * AV + NTHR - 1) / NTHR;  // 16-byte loads per thread and tile
    static_assert(CIN % 8 == 0, "a lane's eight k lie in one tap");
    // The staged inputs share their LDS with the per-wave transposes of the
    // output tiles (bf16 rows of COUT channels, so that outputs leave with
    // 16-byte stores of consecutive channels; after the last tile, the input
    // gradient's channel sums), which take over once every wave's products
    // have read the inputs.  Guard flags of the tile.
    constexpr int OS = 64 + 8;
    constexpr int SAO = TP * AS > WAVES * 32 * OS ? TP * AS : WAVES * 32 * OS;
    __shared__ __attribute__((aligned(16))) uint16_t sW[COUT * RS];
    __shared__ __attribute__((aligned(16))) uint16_t sA[SAO];
    __shared__ uint8_t sG[TPOS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 31, kq = lane >> 5;
    uint16_t *const ow = sA + wave * 32 * OS;  // this wave's output transpose
    // positions tile * TPOS - 2 .. tile * TPOS + TPOS + 1, clamped (both ends
    // of the batch are guard positions, zero)
    uint4 va[NA];
    uint4 vm0, vm1, vm2, vm3;  // MODE 2: the ReLU mask of this wave's 32 positions, 16 bytes a lane
    int vg = 1;
    float gsum[NTILES] = {};  // MODE 2: this lane's sum of g over its rows of every tile, in tile order
    auto fetch = [&](int tile) __attribute__((always_inline)) {
        const int pg = tile * TPOS + (int)threadIdx.x;
        vg = threadIdx.x < TPOS && pg < P ? guard[pg] : 1;
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = threadIdx.x + NTHR * j;
            const int g = e % AV, pp = e / AV;
            int q = tile * TPOS - 2 + pp;
            q = q < 0 ? 0 : (q >= P ? P - 1 : q);
            va[j] = e < TP * AV ? *reinterpret_cast<const uint4 *>(in + (size_t)q * CIN + 8 * g)
                                : make_uint4(0, 0, 0, 0);
        }
    };
    // MODE 2: the ReLU mask of this wave's 32 positions of a tile, fetched
    // when the previous tile's epilogue has consumed the last one
    auto fetch_mask = [&](int tile) __attribute__((always_inline)) {
        if constexpr (MODE == 2) {
            auto ld = [&](int j) {
                const int c = lane + 64 * j, pp = c >> 3, part = c & 7;
                const int p = min(tile * TPOS + wave * 32 + pp, P - 1);
                return *reinterpret_cast<const uint4 *>(mask + (size_t)p * 64 + 8 * part);
            };
            vm0 = ld(0);
            vm1 = ld(1);
            vm2 = ld(2);
            vm3 = ld(3);
        }
    };
    if (blockIdx.x * TPOS < P) {  // in flight while the weights are staged
        fetch(blockIdx.x);
        fetch_mask(blockIdx.x);
    }
    // the weights: every 16-byte load issued before the first LDS write
    constexpr int WV = COUT * ROW / 8, NWV = (WV + NTHR - 1) / NTHR;
    static_assert(ROW % 8 == 0, "a 16-byte piece of weights lies in one row");
    {
        uint4 wv[NWV];
#pragma unroll
        for (int j = 0; j < NWV; ++j) {
            const int e = threadIdx.x + NTHR * j;
            wv[j] = e < WV ? *reinterpret_cast<const uint4 *>(W + 8 * (size_t)e) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < NWV; ++j) {
            const int e = threadIdx.x + NTHR * j;
            if (e < WV) *reinterpret_cast<uint4 *>(&sW[((8 * e) / ROW) * RS + (8 * e) % ROW]) = wv[j];
        }
    }

    for (int tile = blockIdx.x; tile * TPOS < P; tile += gridDim.x) {
        __syncthreads();  // the previous tile's epilogues are done with sA (and sW is staged)
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = threadIdx.x + NTHR * j;
            if (e < TP * AV) *reinterpret_cast<uint4 *>(&sA[(e / AV) * AS + 8 * (e % AV)]) = va[j];
        }
        if (threadIdx.x < TPOS) sG[threadIdx.x] = (uint8_t)vg;
        __syncthreads();
        if ((tile + (int)gridDim.x) * TPOS < P) fetch(tile + gridDim.x);
        const int p0 = tile * TPOS + wave * 32;
        f32x16 acc[NTILES];
#pragma unroll
        for (int nt = 0; nt < NTILES; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[nt][r] = 0.0f;
#pragma unroll
        for (int m = 0; m < KS; ++m) {
            // this half-wave's eight k: tap t, input channels c .. c + 7 of
            // position p0 + i + t - 2, staged at wave * 32 + i + t
            const int k0 = 16 * m + 8 * kq, t = k0 / CIN, c = k0 % CIN;
            const bool tap = t < 5;
            const bf16x8 zero = {};
            const bf16x8 la = *reinterpret_cast<const bf16x8 *>(&sA[(wave * 32 + i + (tap ? t : 0)) * AS + c]);
            const bf16x8 a = tap ? la : zero;
#pragma unroll
            for (int nt = 0; nt < NTILES; ++nt) {
                const bf16x8 lb = *reinterpret_cast<const bf16x8 *>(&sW[(32 * nt + i) * RS + (tap ? k0 : 0)]);
                const bf16x8 b = tap ? lb : zero;
                acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[nt], 0, 0, 0);
            }
        }
        if constexpr (MODE == 1) {
            if (p0 >= P) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int pr = acc_row(r, lane), p = p0 + pr;
                if (p < P && i < NOUT) out_f32[(size_t)p * NOUT + i] = sG[wave * 32 + pr] ? 0.0f : acc[0][r] + bias[i];
            }
        } else {
            __syncthreads();  // every wave's products have read the staged inputs
            if (p0 >= P) continue;
            // 16-byte pieces of the wave's 32 x COUT tile: lane l takes pieces
            // l, l + 64, ... (position piece / 8, channels 8 (piece % 8) ..)
            static_assert(COUT == 64, "the transposed epilogue assumes 64 output channels");
            if constexpr (MODE == 2) {
                // the tile's ReLU mask, as rows of channels
                auto st = [&](int j, const uint4 &v) {
                    const int c = lane + 64 * j, pp = c >> 3, part = c & 7;
                    *reinterpret_cast<uint4 *>(&ow[pp * OS + 8 * part]) = v;
                };
                st(0, vm0);
                st(1, vm1);
                st(2, vm2);
                st(3, vm3);
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int nt = 0; nt < NTILES; ++nt) {
                const int o = 32 * nt + i;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int pr = acc_row(r, lane);
                    const bool g = sG[wave * 32 + pr] != 0;
                    float v = acc[nt][r];
                    if (MODE == 0) v = g ? 0.0f : fmaxf(v + bias[o], 0.0f);
                    else v = (g || !(bf2f(ow[pr * OS + o]) > 0.0f)) ? 0.0f : v;
                    if (MODE == 2) gsum[nt] += v;  // zero at guards and past the batch
                    ow[pr * OS + o] = f2bf(v);  // (pr, o) is this lane's alone
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = lane + 64 * j, pp = c >> 3, part = c & 7, p = p0 + pp;
                if (p < P)
                    *reinterpret_cast<uint4 *>(out_bf16 + (size_t)p * COUT + 8 * part) =
                        *reinterpret_cast<const uint4 *>(&ow[pp * OS + 8 * part]);
            }
            if ((tile + (int)gridDim.x) * TPOS < P) fetch_mask(tile + gridDim.x);
        }
    }
    if constexpr (MODE == 2) {
        // the block's channel sums: lanes of both halves of each wave, then
        // the waves, added in a fixed order (each wave's transpose buffer
        // holds its two halves' sums)
        __syncthreads();
        float *red = reinterpret_cast<float *>(ow);
#pragma unroll
        for (int nt = 0; nt < NTILES; ++nt) red[kq * COUT + 32 * nt + i] = gsum[nt];
        __syncthreads();
        if (threadIdx.x < COUT) {
            float t = 0.0f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const float *rw = reinterpret_cast<const float *>(sA + w * 32 * OS);
                t += rw[threadIdx.x] + rw[COUT + threadIdx.x];
            }
            bsum[(size_t)blockIdx.x * COUT + threadIdx.x] = t;
        }
    }
}

// Partial weight gradient over positions [blockIdx.x * span, ...):
// dW[o][t][i] = sum_p dZ[p][o] X[p + t - 2][i], a GEMM with M = COUT (o),
// N = 5 CIN (t, i) and K = positions.  dZ has ZS channels per position
// (rows o >= ZS are zero).  Each CH-position chunk of dZ and of X (with a
// 2-position halo on each side) is staged transposed in LDS, so a lane's
// eight consecutive positions are adjacent; the chunk is read with 16-byte
// loads (eight channels of a position) one chunk ahead, into registers,
// while the matrix cores work on the current one.
template <int CIN, int COUT, int ZS, int CH, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void dw_mfma(const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ X,
                                               int P, int span, float *__restrict__ partial)
{
    static_assert(CH % 64 == 0, "chunks of whole 16-position steps for both half-waves");
    constexpr int MT = COUT / 32;
    constexpr int NN = 5 * CIN;
    constexpr int NT = (NN + 31) / 32;
    constexpr int TILES = MT * NT;
    constexpr int NTHR = 64 * WAVES;
    constexpr int TPW = (TILES + WAVES - 1) / WAVES;  // output tiles of a wave
    constexpr int ZV = COUT / 8, XV = CIN / 8;  // 8-channel groups
    // staging items: four consecutive positions of one 8-channel group (four
    // 16-byte loads), written as one 8-byte LDS store per channel; the
    // position quads vary fastest across lanes, so that a store instruction
    // covers consecutive positions of a channel row (no bank conflicts)
    constexpr int ZQ = CH / 4, XQ = (CH + 4) / 4;  // position quads: dZ, X (with the halo)
    constexpr int ZI = ZV * ZQ, XI = XV * XQ, NI = (ZI + XI + NTHR - 1) / NTHR;
    static_assert(ZS % 8 == 0 && CIN % 8 == 0, "16-byte groups of channels");
    __shared__ __attribute__((aligned(16))) uint16_t sZ[COUT][CH + 8];
    __shared__ __attribute__((aligned(16))) uint16_t sX[CIN][CH + 8];  // positions p0 - 2 .. p0 + CH + 1

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 31, kq = lane >> 5;
    f32x16 acc[TPW];
#pragma unroll
    for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.0f;

    const int pbeg = blockIdx.x * span, pend = min(P, pbeg + span);
    uint4 vv[NI][4];
    auto fetch = [&](int p0) {
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int u = threadIdx.x + NTHR * j;
            if (u < ZI) {
                const int g = u / ZQ, pq = 4 * (u % ZQ);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int p = p0 + pq + q;
                    vv[j][q] = 8 * g < ZS && p < pend
                                   ? *reinterpret_cast<const uint4 *>(dZ + (size_t)p * ZS + 8 * g)
                                   : make_uint4(0, 0, 0, 0);
                }
            } else if (u < ZI + XI) {
                const int g = (u - ZI) / XQ, pq = 4 * ((u - ZI) % XQ);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    int p = p0 - 2 + pq + q;
                    p = p < 0 ? 0 : (p >= P ? P - 1 : p);
                    vv[j][q] = *reinterpret_cast<const uint4 *>(X + (size_t)p * CIN + 8 * g);
                }
            }
        }
    };
    // channel m of four position vectors -> the row's four consecutive values
    auto quad = [](const uint4 *v, int m) {
        auto word = [&](const uint4 &x) {
            const unsigned d = (m >> 1) == 0 ? x.x : ((m >> 1) == 1 ? x.y : ((m >> 1) == 2 ? x.z : x.w));
            return (m & 1) ? d >> 16 : d & 0xffffu;
        };
        return make_uint2(word(v[0]) | (word(v[1]) << 16), word(v[2]) | (word(v[3]) << 16));
    };
    if (pbeg < pend) fetch(pbeg);
    for (int p0 = pbeg; p0 < pend; p0 += CH) {
        __syncthreads();  // the previous chunk's products have read the LDS tiles
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const int u = threadIdx.x + NTHR * j;
            uint16_t *row = nullptr;
            if (u < ZI) row = &sZ[8 * (u / ZQ)][4 * (u % ZQ)];
            else if (u < ZI + XI) row = &sX[8 * ((u - ZI) / XQ)][4 * ((u - ZI) % XQ)];
            if (row) {
#pragma unroll
                for (int m = 0; m < 8; ++m) *reinterpret_cast<uint2 *>(row + m * (CH + 8)) = quad(vv[j], m);
            }
        }
        __syncthreads();
        if (p0 + CH < pend) fetch(p0 + CH);
#pragma unroll 2
        for (int k16 = 0; k16 < CH; k16 += 16) {
            const int pk = k16 + 8 * kq;
#pragma unroll
            for (int k = 0; k < TPW; ++k) {
                const int tile = wave + WAVES * k;
                if (tile >= TILES) break;
                const int mt = tile % MT, nt = tile / MT;
                const int o = 32 * mt + i;
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&sZ[o][pk]);
                const int n = 32 * nt + i;
                bf16x8 b = {};
                if constexpr (CIN % 32 == 0) {
                    // the tile's 32 columns n lie in one tap t (the same for
                    // the whole wave): two aligned 16-byte reads hold
                    // positions pk .. pk + 15, from which the eight at pk + t
                    // are taken by whole or half-dword shifts
                    const int t = (32 * nt) / CIN, c = n % CIN;
                    const uint4 w0 = *reinterpret_cast<const uint4 *>(&sX[c][pk]);
                    const uint4 w1 = *reinterpret_cast<const uint4 *>(&sX[c][pk + 8]);
                    const unsigned W[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
                    unsigned r[4];
                    switch (t) {
                    case 0:
#pragma unroll
                        for (int q = 0; q < 4; ++q) r[q] = W[q];
                        break;
                    case 1:
#pragma unroll
                        for (int q = 0; q < 4; ++q) r[q] = __builtin_amdgcn_alignbyte(W[q + 1], W[q], 2);
                        break;
                    case 2:
#pragma unroll
                        for (int q = 0; q < 4; ++q) r[q] = W[q + 1];
                        break;
                    case 3:
#pragma unroll
                        for (int q = 0; q < 4; ++q) r[q] = __builtin_amdgcn_alignbyte(W[q + 2], W[q + 1], 2);
                        break;
                    default:
#pragma unroll
                        for (int q = 0; q < 4; ++q) r[q] = W[q + 2];
                        break;
                    }
                    b = __builtin_bit_cast(bf16x8, make_uint4(r[0], r[1], r[2], r[3]));
                } else if (n < NN) {
                    const int t = n / CIN, c = n % CIN;
                    // X[p + t - 2] for p = p0 + pk + j  ->  sX index pk + j + t
#pragma unroll
                    for (int e = 0; e < 8; ++e) b[e] = as_bf(sX[c][pk + t + e]);
                }
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
            }
        }
    }
    float *dst = partial + (size_t)blockIdx.x * COUT * NN;
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int tile = wave + WAVES * k;
        if (tile >= TILES) break;
        const int mt = tile % MT, nt = tile / MT;
        const int n = 32 * nt + i;
        if (n >= NN) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 32 * mt + acc_row(r, lane);
            dst[(size_t)o * NN + n] = acc[k][r];
        }
    }
}

// Sum of count values a[0], a[step], a[2 step], ... added in increasing
// order (deterministic); eight loads are issued before their additions.
__device__ __forceinline__ float ordered_sum(const float *__restrict__ a, int count, size_t step)
{
    float s = 0.0f;
    int k = 0;
    for (; k + 8 <= count; k += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a[(size_t)(k + j) * step];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; k < count; ++k) s += a[(size_t)k * step];
    return s;
}

// dst[e] = sum_b src[b][e], deterministic: the nb slices form kRedGroups
// consecutive groups, each summed in increasing order by its own thread, and
// the group sums are added in group order.  A block holds 256 / kRedGroups
// outputs (consecutive e, so every slice is read coalesced).  One launch
// serves two such reductions (a layer's weight and bias gradients): blocks
// past the first one's take the second.
constexpr int kRedGroups = 8, kRedOutputs = 256 / kRedGroups;
__global__ __launch_bounds__(256) void reduce_partials(RedJob ja, RedJob jb)
{
    __shared__ float part[kRedGroups][kRedOutputs];
    const int ba = (ja.n + kRedOutputs - 1) / kRedOutputs;
    const bool first = (int)blockIdx.x < ba;  // uniform
    const RedJob j = first ? ja : jb;
    const int blk = first ? (int)blockIdx.x : (int)blockIdx.x - ba;
    const int lo = threadIdx.x % kRedOutputs, g = threadIdx.x / kRedOutputs;
    const int e = blk * kRedOutputs + lo;
    const int per = (j.nb + kRedGroups - 1) / kRedGroups;
    const int b0 = min(j.nb, g * per), b1 = min(j.nb, b0 + per);
    part[g][lo] = e < j.n ? ordered_sum(j.src + (size_t)b0 * j.stride + e, b1 - b0, (size_t)j.stride) : 0.0f;
    __syncthreads();
    if (g == 0 && e < j.n) {
        float t = 0.0f;
#pragma unroll
        for (int k = 0; k < kRedGroups; ++k) t += part[k][lo];
        j.dst[e] = t;
    }
}

// bias-gradient partials: per-channel sums of dZ over position slices.  The
// 256 threads form 256 / ZS groups; group k sums positions k, k + groups, ...
// of the slice, then the group sums are added in group order (deterministic).
__global__ __launch_bounds__(256) void db_partial(const float *__restrict__ dZ, int ZS, int P, int span,
                                                  float *__restrict__ partial)
{
    __shared__ float red[256];
    const int groups = 256 / ZS;
    const int o = threadIdx.x % ZS, k = threadIdx.x / ZS;
    const int pbeg = blockIdx.x * span, pend = min(P, pbeg + span);
    const int cnt = pend - pbeg - k > 0 ? (pend - pbeg - k + groups - 1) / groups : 0;
    red[threadIdx.x] = ordered_sum(dZ + (size_t)(pbeg + k) * ZS + o, cnt, (size_t)groups * ZS);
    __syncthreads();
    if (threadIdx.x < ZS) {
        float t = 0.0f;
        for (int g = 0; g < groups; ++g) t += red[g * ZS + o];
        partial[(size_t)blockIdx.x * ZS + o] = t;
    }
}

// squared-error partials and the output-layer gradient dZ (8 channels per
// position, the last six zero)
__global__ __launch_bounds__(256) void loss_grad(const float *__restrict__ out, const float *__restrict__ tgt,
                                                 const uint8_t *__restrict__ guard, int P, float scale,
                                                 float *__restrict__ dZf, uint16_t *__restrict__ dZb,
                                                 float *__restrict__ partial)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        float g0 = 0.0f, g1 = 0.0f;
        if (!guard[p]) {
            const float r0 = out[2 * (size_t)p] - tgt[2 * (size_t)p];
            const float r1 = out[2 * (size_t)p + 1] - tgt[2 * (size_t)p + 1];
            s += r0 * r0 + r1 * r1;
            g0 = 2.0f * r0 * scale;
            g1 = 2.0f * r1 * scale;
        }
        dZf[8 * (size_t)p] = g0;
        dZf[8 * (size_t)p + 1] = g1;
        dZb[8 * (size_t)p] = f2bf(g0);
        dZb[8 * (size_t)p + 1] = f2bf(g1);
#pragma unroll
        for (int c = 2; c < 8; ++c) {
            dZf[8 * (size_t)p + c] = 0.0f;
            dZb[8 * (size_t)p + c] = 0;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam on the FP32 master parameters (c1, c2: bias corrections)
__global__ void adam(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                     float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const float g = grad[e];
        const float mm = b1 * m[e] + (1.0f - b1) * g;
        const float vv = b2 * v[e] + (1.0f - b2) * g * g;
        m[e] = mm;
        v[e] = vv;
        theta[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    }
}

// BF16 copies of every layer's weights (layer blockIdx.y): forward
// Wb[o][t][i] with rows padded to cout_pad, and input-gradient weights
// Wg[i][t][o] = W[o][4 - t][i] with o padded to cin_g (not for layer 0).
__global__ void prep_weights(NetWeightSet w)
{
    const int l = blockIdx.y;
    const float *__restrict__ Wf = w.Wf[l];
    uint16_t *__restrict__ Wb = w.Wb[l];
    uint16_t *__restrict__ Wg = w.Wg[l];
    const int cout = kNetCout[l], cin = kNetCin[l], cout_pad = kNetCoutPad[l], cin_g = kNetGradCin[l];
    const int nf = cout_pad * 5 * cin;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += gridDim.x * blockDim.x) {
        const int o = e / (5 * cin), rem = e % (5 * cin);
        Wb[e] = o < cout ? f2bf(Wf[(size_t)o * 5 * cin + rem]) : (uint16_t)0;
    }
    if (!Wg) return;
    const int ng = cin * 5 * cin_g;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ng; e += gridDim.x * blockDim.x) {
        const int i = e / (5 * cin_g), rem = e % (5 * cin_g);
        const int t = rem / cin_g, o = rem % cin_g;
        Wg[e] = o < cout ? f2bf(Wf[((size_t)o * 5 + (4 - t)) * cin + i]) : (uint16_t)0;
    }
}

// Input features (8 channels, bf16: position, T/T_c, log10 g, form, <rho>,
// height, and the distance to the lever-rule interface at two widths) of one
// column per block, its trailing
// guard positions (block 0 also the two leading ones) and, with a dataset,
// the targets (rho/rho_c - <rho>/rho_c, T/T_c - T_wall/T_c).
__global__ __launch_bounds__(256) void prep(const NetCol *__restrict__ cols, const NetEntry *__restrict__ ent,
                                            const double *__restrict__ rho, const double *__restrict__ T,
                                            double rho_c, double T_c, uint16_t *__restrict__ x,
                                            uint8_t *__restrict__ guard, float *__restrict__ tgt)
{
    const NetEntry e = ent[blockIdx.x];
    const NetCol c = cols[e.src];
    const int H = c.height;
    const uint32_t k1 = f2bf((float)(c.t_reduced - 0.8));
    const uint32_t k2 = f2bf((float)(log10(c.g) + 5.0));
    const uint32_t k3 = f2bf((float)((double)c.form - 1.5));
    const uint32_t k4 = f2bf((float)(c.mean_reduced - 1.3));
    const uint32_t k5 = f2bf((float)((double)H / 2048.0 - 0.5));
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
        const int64_t p = e.pos + y;
        const double yc = (double)y + 0.5, d = yc - c.lever_height;
        const uint32_t k0 = f2bf((float)(yc / (double)H - 0.5));
        const uint32_t k6 = f2bf((float)(fmin(fmax(d / 32.0, -4.0), 4.0) / 4.0));
        const uint32_t k7 = f2bf((float)(fmin(fmax(d / 4.0, -4.0), 4.0) / 4.0));
        *reinterpret_cast<uint4 *>(x + 8 * p) =
            make_uint4(k0 | (k1 << 16), k2 | (k3 << 16), k4 | (k5 << 16), k6 | (k7 << 16));
        guard[p] = 0;
        if (tgt) {
            tgt[2 * p] = (float)(rho[c.offset + y] / rho_c - c.mean_reduced);
            tgt[2 * p + 1] = (float)(T[c.offset + y] / T_c - c.t_reduced);
        }
    }
    // trailing guards pos + H, pos + H + 1; block 0 also the leading pos - 2, pos - 1
    const int j = threadIdx.x;
    if (j < 2 || (j < 4 && blockIdx.x == 0)) {
        const int64_t p = j < 2 ? e.pos + H + j : e.pos - 4 + j;
        *reinterpret_cast<uint4 *>(x + 8 * p) = make_uint4(0u, 0u, 0u, 0u);
        guard[p] = 1;
        if (tgt) tgt[2 * p] = tgt[2 * p + 1] = 0.0f;
    }
}

// Warm-start profiles of one column per block: rho = rho_c (out_0 + <rho>/rho_c)
// shifted so that its mean is <rho>, T = T_c (T_wall/T_c + out_1) with the two
// wall nodes at T_wall.  FP64.
__global__ __launch_bounds__(256) void emit(const NetCol *__restrict__ cols, const NetEntry *__restrict__ ent,
                                            const float *__restrict__ out, double rho_c, double T_c,
                                            double *__restrict__ rho_out, double *__restrict__ T_out)
{
    __shared__ double red[256];
    const NetEntry e = ent[blockIdx.x];
    const NetCol c = cols[e.src];
    const int H = c.height;
    double s = 0.0;
    for (int y = threadIdx.x; y < H; y += blockDim.x)
        s += rho_c * ((double)out[2 * (e.pos + y)] + c.mean_reduced);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double shift = rho_c * c.mean_reduced - red[0] / (double)H;
    const double Tw = T_c * c.t_reduced;
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
        const int64_t p = e.pos + y;
        rho_out[e.out + y] = rho_c * ((double)out[2 * p] + c.mean_reduced) + shift;
        T_out[e.out + y] = (y == 0 || y == H - 1) ? Tw : T_c * (c.t_reduced + (double)out[2 * p + 1]);
    }
}

// raw network outputs of each column, concatenated without guards
__global__ void raw_out(const NetCol *__restrict__ cols, const NetEntry *__restrict__ ent,
                        const float *__restrict__ out, float *__restrict__ dst)
{
    const NetEntry e = ent[blockIdx.x];
    const int H = cols[e.src].height;
    for (int y = threadIdx.x; y < 2 * H; y += blockDim.x) dst[2 * e.out + y] = out[2 * e.pos + y];
}

// one MFMA on caller-provided operands (lane layout check)
__global__ void mfma_probe(const uint16_t *__restrict__ a, const uint16_t *__restrict__ b, float *__restrict__ d)
{
    const int lane = threadIdx.x;
    bf16x8 av, bv;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        av[k] = as_bf(a[lane * 8 + k]);
        bv[k] = as_bf(b[lane * 8 + k]);
    }
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) d[lane * 16 + r] = acc[r];
}

// persistent convolution grid: blocks of kConvWaves waves on tiles of
// 32 kConvWaves positions, at most two blocks per compute unit
constexpr int kConvWaves = 8, kConvTile = 32 * kConvWaves, kConvBlocks = 512;
unsigned conv_blocks(int64_t P)
{
    const int64_t t = (P + kConvTile - 1) / kConvTile;
    return (unsigned)(t < kConvBlocks ? t : kConvBlocks);
}

// waves of a weight-gradient block (they share the staged chunks and split
// the output tiles): 16 for long slices, 8 for short ones
constexpr int kDwWavesBig = 16, kDwWavesSmall = 8;

// slice length (a multiple of 64 positions) and slice count for nblocks
void slices(int64_t P, int nblocks, int *span, int *nb)
{
    int64_t s = (P + nblocks - 1) / nblocks;
    s = (s + 63) / 64 * 64;
    *span = (int)s;
    *nb = (int)((P + s - 1) / s);
}

}  // namespace

hipError_t net_prep(const NetCol *cols, const NetEntry *entries, int n, const double *rho, const double *T,
                    double rho_c, double T_c, uint16_t *x, uint8_t *guard, float *tgt, hipStream_t s)
{
    hipLaunchKernelGGL(prep, dim3(n), dim3(256), 0, s, cols, entries, rho, T, rho_c, T_c, x, guard, tgt);
    return hipGetLastError();
}

hipError_t net_emit(const NetCol *cols, const NetEntry *entries, int n, const float *out, double rho_c,
                    double T_c, double *rho_out, double *T_out, hipStream_t s)
{
    hipLaunchKernelGGL(emit, dim3(n), dim3(256), 0, s, cols, entries, out, rho_c, T_c, rho_out, T_out);
    return hipGetLastError();
}

hipError_t net_raw_out(const NetCol *cols, const NetEntry *entries, int n, const float *out, float *dst,
                       hipStream_t s)
{
    hipLaunchKernelGGL(raw_out, dim3(n), dim3(256), 0, s, cols, entries, out, dst);
    return hipGetLastError();
}

hipError_t net_conv_forward(int layer, const uint16_t *in, const uint16_t *W, const float *bias, int64_t P,
                            const uint8_t *guard, uint16_t *out_bf16, float *out_f32, hipStream_t s)
{
    const dim3 g(conv_blocks(P)), b(64 * kConvWaves);
    const int p = (int)P;
    if (layer == 0)
        hipLaunchKernelGGL((conv_mfma<8, 2, 0, 64, kConvWaves>), g, b, 0, s, in, W, bias, p, guard, nullptr, nullptr, out_bf16,
                           nullptr);
    else if (layer < 5)
        hipLaunchKernelGGL((conv_mfma<64, 2, 0, 64, kConvWaves>), g, b, 0, s, in, W, bias, p, guard, nullptr, nullptr, out_bf16,
                           nullptr);
    else
        hipLaunchKernelGGL((conv_mfma<64, 1, 1, 2, kConvWaves>), g, b, 0, s, in, W, bias, p, guard, nullptr, out_f32, nullptr,
                           nullptr);
    return hipGetLastError();
}

hipError_t net_conv_input_grad(int layer, const uint16_t *dZ, const uint16_t *Wg, int64_t P, const uint8_t *guard,
                               const uint16_t *act_in, uint16_t *dprev_bf16, float *bsum, int *nbsum, hipStream_t s)
{
    const unsigned nb = conv_blocks(P);
    const dim3 g(nb), b(64 * kConvWaves);
    const int p = (int)P;
    if (layer == 5)
        hipLaunchKernelGGL((conv_mfma<8, 2, 2, 64, kConvWaves>), g, b, 0, s, dZ, Wg, nullptr, p, guard, act_in, nullptr,
                           dprev_bf16, bsum);
    else
        hipLaunchKernelGGL((conv_mfma<64, 2, 2, 64, kConvWaves>), g, b, 0, s, dZ, Wg, nullptr, p, guard, act_in, nullptr,
                           dprev_bf16, bsum);
    *nbsum = (int)nb;
    return hipGetLastError();
}

hipError_t net_weight_grad(int layer, const uint16_t *dZ, const uint16_t *X, int64_t P, int nblocks,
                           float *partial, float *dW, const RedJob &bias, hipStream_t s)
{
    int span, nb;
    slices(P, nblocks, &span, &nb);
    const int p = (int)P;
    // long slices: 128-position chunks (half the per-chunk barriers, twice
    // the time for each chunk's loads to arrive) on 16 waves; short slices:
    // 64-position chunks on 8 waves (256 columns of 1024: 0.62 -> 0.52 ms per
    // step; the 32-column training batches would lose 6-9% with either)
    const bool big = span >= 512;
    const dim3 th(64 * (big ? kDwWavesBig : kDwWavesSmall));
    int stride;
    if (layer == 0) {
        stride = 64 * 5 * 8;
        auto k = big ? dw_mfma<8, 64, 64, 128, kDwWavesBig> : dw_mfma<8, 64, 64, 64, kDwWavesSmall>;
        hipLaunchKernelGGL(k, dim3(nb), th, 0, s, dZ, X, p, span, partial);
    } else if (layer < 5) {
        stride = 64 * 5 * 64;
        auto k = big ? dw_mfma<64, 64, 64, 128, kDwWavesBig> : dw_mfma<64, 64, 64, 64, kDwWavesSmall>;
        hipLaunchKernelGGL(k, dim3(nb), th, 0, s, dZ, X, p, span, partial);
    } else {
        stride = 32 * 5 * 64;  // rows 2..31 are zero padding
        auto k = big ? dw_mfma<64, 32, 8, 128, kDwWavesBig> : dw_mfma<64, 32, 8, 64, kDwWavesSmall>;
        hipLaunchKernelGGL(k, dim3(nb), th, 0, s, dZ, X, p, span, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the weight gradient from the slices' partials and, in the same
    // launch, the bias gradient from its partials
    const RedJob w{partial, nb, stride, kNetCout[layer] * 5 * kNetCin[layer], dW};
    const int blocks = (w.n + kRedOutputs - 1) / kRedOutputs + (bias.n + kRedOutputs - 1) / kRedOutputs;
    hipLaunchKernelGGL(reduce_partials, dim3(blocks), dim3(256), 0, s, w, bias);
    return hipGetLastError();
}

hipError_t net_bias_partials(int zs, const float *dZ, int64_t P, int nblocks, float *partial, int *nparts,
                             hipStream_t s)
{
    int span, nb;
    slices(P, nblocks, &span, &nb);
    hipLaunchKernelGGL(db_partial, dim3(nb), dim3(256), 0, s, dZ, zs, (int)P, span, partial);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t net_loss(const float *out, const float *tgt, const uint8_t *guard, int64_t P, float scale, float *dZf,
                    uint16_t *dZb, float *partial, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(loss_grad, dim3(nblocks), dim3(256), 0, s, out, tgt, guard, (int)P, scale, dZf, dZb,
                       partial);
    return hipGetLastError();
}

hipError_t net_adam(float *theta, const float *grad, float *m, float *v, int n, float lr, float b1, float b2,
                    float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(adam, dim3((n + 255) / 256), dim3(256), 0, s, theta, grad, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t net_prep_weights(const NetWeightSet &w, hipStream_t s)
{
    hipLaunchKernelGGL(prep_weights, dim3(80, kNetLayers), dim3(256), 0, s, w);
    return hipGetLastError();
}

hipError_t net_mfma_probe(const uint16_t *a, const uint16_t *b, float *d, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_probe, dim3(1), dim3(64), 0, s, a, b, d);
    return hipGetLastError();
}

}  // namespace tplbm
