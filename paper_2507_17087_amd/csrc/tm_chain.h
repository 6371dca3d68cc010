// tm_chain.h -- device functions shared by the kernels: evaluation of the
// transformation chain for one final-space coordinate, per-coordinate projection.
#pragma once

#include <hip/hip_runtime.h>

#include "tm_internal.h"

namespace tmk {

// Copy a DevCand into LDS with all threads of the block (it is read many times).
__device__ __forceinline__ void stage_cand(DevCand* dst, const DevCand* src) {
    const int32_t* s = reinterpret_cast<const int32_t*>(src);
    int32_t* d = reinterpret_cast<int32_t*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(DevCand) / 4); i += blockDim.x) d[i] = s[i];
}

// floor(a / b) and a mod b for a >= 0, b >= 1: a 32-bit division when both operands
// fit in 32 bits (nearly always), else the 64-bit one.
__device__ __forceinline__ int64_t div_nn(int64_t a, int64_t b) {
    if ((((uint64_t)a | (uint64_t)b) >> 32) == 0) return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}
__device__ __forceinline__ int64_t mod_nn(int64_t a, int64_t b) {
    if ((((uint64_t)a | (uint64_t)b) >> 32) == 0) return (int64_t)((uint32_t)a % (uint32_t)b);
    return a % b;
}

// A value that is the same in every lane of the wave, moved to a scalar register.
__device__ __forceinline__ int32_t wave_uniform(int32_t x) {
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}
__device__ __forceinline__ int64_t wave_uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Owner key of final-space coordinate v: undo the ops on the linear index (C order)
// of the processor space, last op first, down to Machine(GPU) = (nodes, gpus).  An
// op touches a contiguous range of dims: with lo the product of the dims after the
// range, the index is (h * W + x) * lo + l0, where x indexes the range (W its
// volume); the op maps x between its output and input digits, and h, l0 pass
// through.  Every index stays below the processor-space volume (<= 2^24), so the
// arithmetic is 32-bit; the descriptor c must be the same in every lane of the
// wave (its fields are then scalars).
__device__ inline int32_t owner_key(const DevCand& c, int32_t v) {
    uint32_t L = (uint32_t)v;
    const int nops = wave_uniform(c.nops);
    for (int t = nops - 1; t >= 0; --t) {
        const int kind = wave_uniform(c.op_kind[t]);
        const uint32_t lo = (uint32_t)wave_uniform(c.inv_lo[t]), wi = (uint32_t)wave_uniform(c.inv_win[t]),
                       wo = (uint32_t)wave_uniform(c.inv_wout[t]);
        const uint32_t q = L / lo, l0 = L - q * lo;
        const uint32_t h = q / wo;
        uint32_t x = q - h * wo, m;
        if (kind == TM_SPLIT || kind == TM_BALANCE_SPLIT) {
            // output digits (a, a1) of extents (b, c), x = a * c + a1; input a + a1 * b
            const uint32_t pb = (uint32_t)wave_uniform(c.op_b[t]), cc = (uint32_t)wave_uniform(c.inv_c[t]);
            const uint32_t a = x / cc, a1 = x - a * cc;
            const uint32_t vv = a + a1 * pb;
            // balance_split folds vv in [0, b * c) onto the input extent (wi <= b * c)
            m = kind == TM_SPLIT ? vv : (uint32_t)div_nn((int64_t)vv * wi, (int64_t)wo);
        } else if (kind == TM_MERGE) {
            // output (a of extent s_pa * s_pb, mid); input (a mod s_pa, mid, a / s_pa)
            const int pa = wave_uniform(c.op_a[t]), pb = wave_uniform(c.op_b[t]);
            const uint32_t mid = (uint32_t)wave_uniform(c.inv_mid[t]);
            const uint32_t spa = (uint32_t)wave_uniform(c.shape[t][pa]), spb = (uint32_t)wave_uniform(c.shape[t][pb]);
            const uint32_t a = x / mid, xm = x - a * mid;
            const uint32_t ahi = a / spa, alo = a - ahi * spa;
            m = (alo * mid + xm) * spb + ahi;
        } else if (kind == TM_SWAP) {
            // output (y_lo of extent s_hi, mid, y_hi of extent s_lo); input (y_hi, mid, y_lo)
            const int pa = wave_uniform(c.op_a[t]), pb = wave_uniform(c.op_b[t]);
            const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
            const uint32_t mid = (uint32_t)wave_uniform(c.inv_mid[t]);
            const uint32_t slo = (uint32_t)wave_uniform(c.shape[t][plo]), shi = (uint32_t)wave_uniform(c.shape[t][phi]);
            const uint32_t ms = mid * slo;
            const uint32_t ylo = x / ms, rest = x - ylo * ms;
            const uint32_t xm = rest / slo, yhi = rest - xm * slo;
            m = (yhi * mid + xm) * shi + ylo;
        } else {  // TM_DECOMPOSE: output digits of extents f[0..k) in C order; input little-endian
            const int k = wave_uniform(c.op_nf[t]);
            uint32_t dg[TM_MAX_LRANK] = {0, 0, 0, 0}, f[TM_MAX_LRANK] = {1, 1, 1, 1};
#pragma unroll
            for (int j = 0; j < TM_MAX_LRANK; ++j) f[j] = j < k ? (uint32_t)wave_uniform(c.op_f[t][j]) : 1u;
#pragma unroll
            for (int j = TM_MAX_LRANK - 1; j >= 0; --j) {
                if (j < k) {
                    const uint32_t qq = x / f[j];
                    dg[j] = x - qq * f[j];
                    x = qq;
                }
            }
            m = 0;
#pragma unroll
            for (int j = TM_MAX_LRANK - 1; j >= 0; --j) m = j < k ? m * f[j] + dg[j] : m;
        }
        L = (h * wi + m) * lo + l0;
    }
    const uint32_t g = (uint32_t)wave_uniform(c.gpus);
    const uint32_t node = L / g;
    return (int32_t)((node << wave_uniform(c.gbits)) | (L - node * g));
}

// Contribution of coordinate x of launch dim d to the linear final index.
__device__ inline int32_t coord_value(const DevCand& c, int d, int64_t x) {
    int32_t v = 0;
    for (int j = 0; j < c.frank; ++j) {
        if (c.proj_src[j] != d) continue;
        const int64_t s = c.fshape[j];
        const int64_t a = c.proj_mode[j] == TM_BLOCK ? div_nn(x * s, c.extent[d]) : mod_nn(x, s);
        v += (int32_t)a * c.fstride[j];
    }
    return v;
}

}  // namespace tmk
