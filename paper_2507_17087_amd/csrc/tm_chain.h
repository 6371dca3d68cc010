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

// Barrier of a workgroup of nw waves, for data passed through LDS.  A one-wave
// workgroup needs no s_barrier: its LDS accesses execute in program order, so a
// wavefront fence (which also keeps the compiler from moving them) suffices, and it
// does not wait for the wave's global memory traffic, as __syncthreads does.
__device__ __forceinline__ void lds_sync(int nw) {
    if (nw > 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// floor(n / d) for n < 2^24 and 1 <= d <= 2^24, given r = 1 / d rounded to the
// nearest float.  For d >= 2 the quotient n / d is below 2^23, and the float product
// n * r (two roundings of relative size 2^-24 each) is within 1 of it, so its
// truncation is the quotient or one off either way, which the remainder test
// corrects; d = 1 and d = 2^24 are exact.  q * d < 2^25, and 24-bit operands are
// exact in the 24-bit multiply (d = 2^24 only occurs with q = 0).
__device__ __forceinline__ uint32_t div24(uint32_t n, uint32_t d, float r) {
    const uint32_t q = (uint32_t)((float)n * r);
    const int32_t rem = (int32_t)(n - __umul24(q, d));
    return rem < 0 ? q - 1 : (rem >= (int32_t)d ? q + 1 : q);
}

// Reciprocals of the divisors the inverse chain uses (the quotient estimates of
// div24), computed once per candidate: for op t, rt[8t] = 1 / inv_lo, rt[8t + 1] =
// 1 / inv_wout, then split / balance_split: 1 / inv_c; merge: 1 / inv_mid, 1 / s_pa;
// swap: 1 / (inv_mid * s_lo), 1 / s_lo; decompose: rt[8t + 4 + j] = 1 / f_j; unused
// slots 1.  rt[kRecipGpus] = 1 / gpus, rt[kRecipFinal + j] = 1 / (final extent j).
// Threads tid of nt each take slots.
constexpr int kRecipGpus = 8 * TM_MAX_OPS, kRecipFinal = kRecipGpus + 1, kRecipSlots = kRecipFinal + TM_MAX_MRANK;
__device__ inline void op_reciprocals(const DevCand& c, float* rt, int tid, int nt) {
    for (int e = tid; e < kRecipSlots; e += nt) {
        uint32_t d = 1;
        if (e == kRecipGpus) {
            d = (uint32_t)c.gpus;
        } else if (e >= kRecipFinal) {
            d = e - kRecipFinal < c.frank ? (uint32_t)c.fshape[e - kRecipFinal] : 1u;
        } else {
            const int t = e >> 3, sl = e & 7;
            if (t < c.nops) {
                const int kind = c.op_kind[t], pa = c.op_a[t], pb = c.op_b[t];
                const int plo = pa < pb ? pa : pb;
                if (sl == 0) d = (uint32_t)c.inv_lo[t];
                else if (sl == 1) d = (uint32_t)c.inv_wout[t];
                else if (kind == TM_SPLIT || kind == TM_BALANCE_SPLIT) d = sl == 2 ? (uint32_t)c.inv_c[t] : 1u;
                else if (kind == TM_MERGE) d = sl == 2 ? (uint32_t)c.inv_mid[t] : (sl == 3 ? (uint32_t)c.shape[t][pa] : 1u);
                else if (kind == TM_SWAP)
                    d = sl == 2 ? (uint32_t)c.inv_mid[t] * (uint32_t)c.shape[t][plo] : (sl == 3 ? (uint32_t)c.shape[t][plo] : 1u);
                else if (sl >= 4 && sl - 4 < c.op_nf[t]) d = (uint32_t)c.op_f[t][sl - 4];
            }
        }
        rt[e] = 1.0f / (float)d;
    }
}

// Owner keys of final-space coordinates v0 + tid, v0 + tid + nt, ... below v1
// (tid, nt: the thread's index and count), written (AND keep) to out[v - vbase].
// Each key undoes the ops on the linear index (C order) of the processor space,
// last op first, down to Machine(GPU) = (nodes, gpus).  An op touches a contiguous
// range of dims: with lo the product of the dims after the range, the index is
// (h * W + x) * lo + l0, where x indexes the range (W its volume); the op maps x
// between its output and input digits, and h, l0 pass through.  Every index stays
// below the processor-space volume (<= 2^24).  A thread takes KPT coordinates per
// pass through the ops, so each op's constants are read once per pass; rt holds the
// divisors' reciprocals (op_reciprocals).  The descriptor c must be the same in every
// lane of the wave (its fields are then scalars).
template <int KPT>
__device__ inline void owner_keys(const DevCand& c, const float* __restrict__ rt, int32_t* __restrict__ out,
                                  int32_t vbase, int32_t v0, int32_t v1, int32_t keep, int tid, int nt) {
    const int nops = wave_uniform(c.nops);
    const uint32_t g = (uint32_t)wave_uniform(c.gpus);
    const int gb = wave_uniform(c.gbits);
    const float rg = rt[kRecipGpus];
    for (int32_t base = v0 + tid; base < v1; base += KPT * nt) {
        uint32_t L[KPT];
#pragma unroll
        for (int i = 0; i < KPT; ++i) {
            const int32_t v = base + i * nt;
            L[i] = (uint32_t)(v < v1 ? v : v1 - 1);  // out-of-range slots repeat a valid index
        }
        for (int t = nops - 1; t >= 0; --t) {
            const int kind = wave_uniform(c.op_kind[t]);
            const uint32_t lo = (uint32_t)wave_uniform(c.inv_lo[t]), wi = (uint32_t)wave_uniform(c.inv_win[t]),
                           wo = (uint32_t)wave_uniform(c.inv_wout[t]);
            const float* r = rt + 8 * t;
            const float rlo = r[0], rwo = r[1];
            if (kind == TM_SPLIT || kind == TM_BALANCE_SPLIT) {
                // output digits (a, a1) of extents (b, c), x = a * c + a1; input a + a1 * b;
                // balance_split folds that onto the input extent (wi <= b * c)
                const uint32_t pb = (uint32_t)wave_uniform(c.op_b[t]), cc = (uint32_t)wave_uniform(c.inv_c[t]);
                const float rc = r[2];
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const uint32_t q = div24(L[i], lo, rlo), l0 = L[i] - __umul24(q, lo);
                    const uint32_t h = div24(q, wo, rwo), x = q - __umul24(h, wo);
                    const uint32_t aa = div24(x, cc, rc), a1 = x - __umul24(aa, cc);
                    const uint32_t vv = aa + __umul24(a1, pb);
                    const uint32_t m = kind == TM_SPLIT ? vv : (uint32_t)div_nn((int64_t)vv * wi, (int64_t)wo);
                    L[i] = __umul24(__umul24(h, wi) + m, lo) + l0;
                }
            } else if (kind == TM_MERGE) {
                // output (a of extent s_pa * s_pb, mid); input (a mod s_pa, mid, a / s_pa)
                const int pa = wave_uniform(c.op_a[t]), pb = wave_uniform(c.op_b[t]);
                const uint32_t mid = (uint32_t)wave_uniform(c.inv_mid[t]);
                const uint32_t spa = (uint32_t)wave_uniform(c.shape[t][pa]), spb = (uint32_t)wave_uniform(c.shape[t][pb]);
                const float rmid = r[2], rspa = r[3];
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const uint32_t q = div24(L[i], lo, rlo), l0 = L[i] - __umul24(q, lo);
                    const uint32_t h = div24(q, wo, rwo), x = q - __umul24(h, wo);
                    const uint32_t aa = div24(x, mid, rmid), xm = x - __umul24(aa, mid);
                    const uint32_t ahi = div24(aa, spa, rspa), alo = aa - __umul24(ahi, spa);
                    const uint32_t m = __umul24(__umul24(alo, mid) + xm, spb) + ahi;
                    L[i] = __umul24(__umul24(h, wi) + m, lo) + l0;
                }
            } else if (kind == TM_SWAP) {
                // output (y_lo of extent s_hi, mid, y_hi of extent s_lo); input (y_hi, mid, y_lo)
                const int pa = wave_uniform(c.op_a[t]), pb = wave_uniform(c.op_b[t]);
                const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
                const uint32_t mid = (uint32_t)wave_uniform(c.inv_mid[t]);
                const uint32_t slo = (uint32_t)wave_uniform(c.shape[t][plo]), shi = (uint32_t)wave_uniform(c.shape[t][phi]);
                const uint32_t ms = mid * slo;
                const float rms = r[2], rslo = r[3];
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const uint32_t q = div24(L[i], lo, rlo), l0 = L[i] - __umul24(q, lo);
                    const uint32_t h = div24(q, wo, rwo), x = q - __umul24(h, wo);
                    const uint32_t ylo = div24(x, ms, rms), rest = x - __umul24(ylo, ms);
                    const uint32_t xm = div24(rest, slo, rslo), yhi = rest - __umul24(xm, slo);
                    const uint32_t m = __umul24(__umul24(yhi, mid) + xm, shi) + ylo;
                    L[i] = __umul24(__umul24(h, wi) + m, lo) + l0;
                }
            } else {  // TM_DECOMPOSE: output digits of extents f[0..k) in C order; input little-endian
                const int k = wave_uniform(c.op_nf[t]);
                uint32_t f[TM_MAX_LRANK];
                float rf[TM_MAX_LRANK];
#pragma unroll
                for (int j = 0; j < TM_MAX_LRANK; ++j) {
                    f[j] = j < k ? (uint32_t)wave_uniform(c.op_f[t][j]) : 1u;
                    rf[j] = r[4 + j];
                }
#pragma unroll
                for (int i = 0; i < KPT; ++i) {
                    const uint32_t q = div24(L[i], lo, rlo), l0 = L[i] - __umul24(q, lo);
                    const uint32_t h = div24(q, wo, rwo);
                    uint32_t x = q - __umul24(h, wo);
                    uint32_t dg[TM_MAX_LRANK];
#pragma unroll
                    for (int j = TM_MAX_LRANK - 1; j >= 0; --j) {
                        const uint32_t qq = j < k ? div24(x, f[j], rf[j]) : x;
                        dg[j] = x - __umul24(qq, f[j]);
                        x = qq;
                    }
                    uint32_t m = 0;
#pragma unroll
                    for (int j = TM_MAX_LRANK - 1; j >= 0; --j) m = j < k ? __umul24(m, f[j]) + dg[j] : m;
                    L[i] = __umul24(__umul24(h, wi) + m, lo) + l0;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < KPT; ++i) {
            const int32_t v = base + i * nt;
            if (v < v1) {
                const uint32_t node = div24(L[i], g, rg);
                out[v - vbase] = (int32_t)((node << gb) | (L[i] - __umul24(node, g))) & keep;
            }
        }
    }
}

// owner_keys with the keys per thread chosen by the range's length: slots past the
// range repeat its last index, so a range of at most nt (2 nt) coordinates takes one
// (two) per thread.  The length is the same in every lane.
__device__ inline void owner_keys_sized(const DevCand& c, const float* __restrict__ rt, int32_t* __restrict__ out,
                                        int32_t vbase, int32_t v0, int32_t v1, int32_t keep, int tid, int nt) {
    const int32_t len = v1 - v0;
    if (len <= nt) owner_keys<1>(c, rt, out, vbase, v0, v1, keep, tid, nt);
    else if (len <= 2 * nt) owner_keys<2>(c, rt, out, vbase, v0, v1, keep, tid, nt);
    else owner_keys<4>(c, rt, out, vbase, v0, v1, keep, tid, nt);
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
