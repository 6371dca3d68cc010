// tm_ranker.h -- internal interface of the learned ranker (kernels <-> host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tm_internal.h"

namespace tmk {

constexpr int kFeat = 64;    // features per candidate
constexpr int kWidth = 256;  // hidden width (three hidden layers)
constexpr int kOut = 2;      // heads: log2(1 + bytes), log2(1 + inter-node bytes), standardised
constexpr int kSplits = 32;  // row splits of the weight-gradient reductions

// Offsets (in floats) of each tensor in the flat fp32 parameter vector.
struct RankerLayout {
    int64_t w1, b1, w2, b2, w3, b3, w4, b4, count;
};

constexpr RankerLayout ranker_layout() {
    RankerLayout L{};
    L.w1 = 0;                              // [kFeat][kWidth] row-major (in, out)
    L.b1 = L.w1 + kFeat * kWidth;          // [kWidth]
    L.w2 = L.b1 + kWidth;                  // [kWidth][kWidth]
    L.b2 = L.w2 + kWidth * kWidth;
    L.w3 = L.b2 + kWidth;                  // [kWidth][kWidth]
    L.b3 = L.w3 + kWidth * kWidth;
    L.w4 = L.b3 + kWidth;                  // [kWidth][kOut]
    L.b4 = L.w4 + kWidth * kOut;           // [kOut]
    L.count = L.b4 + kOut;
    return L;
}

// Device views of the weights: bf16 copies row-major (w*) and transposed (w*t);
// biases are read from the fp32 master vector.
struct RankerWeights {
    uint16_t *w1, *w1t, *w2, *w2t, *w3, *w3t, *w4;
    const float *b1, *b2, *b3, *b4;
    RankerLayout layout;
};

// Writes the bf16 copies of master parameter i.
__device__ __forceinline__ void publish_param(int64_t i, float v, const RankerWeights& W) {
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    const uint16_t h = (uint16_t)(u >> 16);
    const RankerLayout& L = W.layout;
    if (i >= L.w1 && i < L.b1) {
        const int64_t j = i - L.w1, r = j / kWidth, c = j % kWidth;
        W.w1[j] = h;
        W.w1t[c * kFeat + r] = h;
    } else if (i >= L.w2 && i < L.b2) {
        const int64_t j = i - L.w2, r = j / kWidth, c = j % kWidth;
        W.w2[j] = h;
        W.w2t[c * kWidth + r] = h;
    } else if (i >= L.w3 && i < L.b3) {
        const int64_t j = i - L.w3, r = j / kWidth, c = j % kWidth;
        W.w3[j] = h;
        W.w3t[c * kWidth + r] = h;
    } else if (i >= L.w4 && i < L.b4) {
        W.w4[i - L.w4] = h;
    }
}

// Per-batch work buffers of training.
struct RankerBuffers {
    uint16_t *X, *H1, *H2, *H3, *dH1, *dH2, *dH3;  // bf16 [rows][width]
    float *Y, *T, *dY;                             // fp32 [rows][kOut]
    float* grad;                                   // fp32 [count]
    float* part;                                   // fp32 [kSplits][kWidth * kWidth]
};

constexpr int kMaxMrankCross = 8;  // node-crossing fractions kept per candidate
// The descriptor estimate of the ghost cells enters the features as
// log2(1 + est) / kBaseScale at kBaseFeat[0] (feature kBaseFeat[1], the inter-node
// head's base, is 0); the network learns the residual of log2(1 + exact bytes) over
// kBaseScale * feature, so the estimate keeps its fp32 precision instead of passing
// through bf16.
constexpr int kBaseFeat[kOut] = {23, 60};
constexpr float kBaseScale = 32.f;
// Per-candidate chain statistics: 2 * kMaxMrankCross floats, then 2 doubles (estimates).
constexpr int64_t kCrossFloats = 2 * kMaxMrankCross;
inline double* chain_estimates(float* cross, int64_t n) {
    return reinterpret_cast<double*>(cross + n * kCrossFloats);  // 64n bytes in: 8-byte aligned
}

// Features of n candidates: bf16 rows X, fp32 copies f32 (nullable), and the
// descriptor estimate est[2i] (est[2i+1] = 0).
hipError_t launch_features(const DevCand* cands, int64_t n, const int32_t* d_halo, double* est, uint16_t* X,
                           float* f32, hipStream_t s);
// Chain statistics and block-model estimates of entries 0..n-1: candidate idx[i]
// (negative: skipped) or i without idx; outputs at entry i of cross and
// chain_estimates(cross, n).
hipError_t launch_chain_stats(const DevCand* cands, const int64_t* idx, int64_t n, int32_t max_vol,
                              const int32_t* d_halo, float* cross, hipStream_t s);
hipError_t launch_mlp_forward(const uint16_t* X, int64_t n, const RankerWeights& W, float* Y, uint16_t* H1,
                              uint16_t* H2, uint16_t* H3, hipStream_t s);
hipError_t launch_backward(const RankerBuffers& B, const RankerWeights& W, int64_t n, float s0, float s1,
                           hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, int64_t t, const RankerWeights& W, hipStream_t s);
hipError_t launch_publish(const float* p, int64_t count, const RankerWeights& W, hipStream_t s);
// The k smallest (score, index) entries of each segment (k_select): sel[s*k ..)
// in index order, -1 after; stride > 0 takes segment s as the first
// min(stride, seg[s+1] - seg[s]) entries from s * stride; remap (nullable) maps an
// entry to the index written.
hipError_t launch_select(const float* score, const int64_t* seg, int64_t nseg, int64_t stride, int k, float margin,
                         const int64_t* remap, int64_t* sel, hipStream_t s);
// Scores from the heads Y (nullable: the estimates alone) and the estimates est.
hipError_t launch_combine(const float* Y, const double* est, int64_t n, const float* mu, const float* sigma,
                          float lambda, float* s, hipStream_t st);
// The sub-batch of the selected candidates (sel[nsel], -1 skipped); sizes: scratch
// of 2 * nsel int64 (their table words and counting items).
hipError_t launch_gather(const DevCand* cands, const int64_t* sel, int64_t nsel, int k, int64_t cells_per_item,
                         DevCand* sub, int64_t* map, int64_t* seg_out, DevHeader* hdr, const DevHeader* proto,
                         int64_t* sizes, hipStream_t s);
hipError_t launch_map_best(const int64_t* sub_best, const int64_t* seg, const int64_t* map,
                           const tm_stencil_cost* sub_cost, int64_t nseg, const int64_t* orig_seg, int64_t* best,
                           tm_stencil_cost* best_cost, hipStream_t s);
hipError_t launch_pick_costs(const int64_t* best, const int64_t* seg, const tm_stencil_cost* cost, int64_t nseg,
                             tm_stencil_cost* best_cost, hipStream_t s);

}  // namespace tmk
