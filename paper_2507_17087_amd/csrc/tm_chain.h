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

// Owner key of final-space coordinate v: decode v (C order), then undo the ops.
__device__ inline int32_t owner_key(const DevCand& c, int32_t v) {
    int32_t a[TM_MAX_MRANK], b[TM_MAX_MRANK];
    for (int j = c.frank - 1; j >= 0; --j) {
        const int32_t s = c.fshape[j];
        a[j] = v % s;
        v /= s;
    }
    for (int t = c.nops - 1; t >= 0; --t) {
        const int r = c.rank[t];
        const int32_t* s = c.shape[t];
        const int pa = c.op_a[t], pb = c.op_b[t];
        switch (c.op_kind[t]) {
            case TM_SPLIT:
                for (int u = 0; u < pa; ++u) b[u] = a[u];
                b[pa] = a[pa] + a[pa + 1] * pb;
                for (int u = pa + 1; u < r; ++u) b[u] = a[u + 1];
                break;
            case TM_MERGE:
                for (int u = 0; u < r; ++u) {
                    if (u < pa || (u > pa && u < pb)) b[u] = a[u];
                    else if (u == pa) b[u] = a[pa] % s[pa];
                    else if (u == pb) b[u] = a[pa] / s[pa];
                    else b[u] = a[u - 1];
                }
                break;
            case TM_SWAP:
                for (int u = 0; u < r; ++u) b[u] = a[u];
                b[pa] = a[pb];
                b[pb] = a[pa];
                break;
            case TM_BALANCE_SPLIT: {
                const int64_t si = s[pa];
                const int64_t cc = div_nn(si + pb - 1, pb);
                const int64_t vv = (int64_t)a[pa] + (int64_t)a[pa + 1] * pb;
                for (int u = 0; u < pa; ++u) b[u] = a[u];
                b[pa] = (int32_t)div_nn(vv * si, (int64_t)pb * cc);
                for (int u = pa + 1; u < r; ++u) b[u] = a[u + 1];
                break;
            }
            default: {  // TM_DECOMPOSE
                const int k = c.op_nf[t];
                int32_t acc = 0;
                for (int m = k - 1; m >= 0; --m) acc = acc * c.op_f[t][m] + a[pa + m];
                for (int u = 0; u < pa; ++u) b[u] = a[u];
                b[pa] = acc;
                for (int u = pa + 1; u < r; ++u) b[u] = a[u + k - 1];
                break;
            }
        }
        for (int u = 0; u < r; ++u) a[u] = b[u];
    }
    return (a[0] << c.gbits) | a[1];
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
