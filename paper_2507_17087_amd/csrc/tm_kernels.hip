// tm_kernels.hip -- gfx950 kernels of libtaskmap.
//
// Data layout.  For each candidate the table-build kernel writes, into a device
// arena, (1) the chain table T[v]: the owner of every coordinate v of the final
// processor space (C order), found by inverting the transformation chain last to
// first (Fig. 6 formulas, decompose as composed splits per Sec. 4.2, balance_split
// as the fold described in taskmap.h), stored as the key (node << gbits) | gpu so
// that owner identity and node are both one integer operation away; and (2) one
// coordinate table per launch dim d: C_d[x] = sum over final dims j projected
// from d of a_j(x) * stride_j (block: floor(x*s_j/l_d), cyclic: x mod s_j), with
// the number of distinct non-zero index offsets to the star neighbours within the
// halo along d in bits 24..27 (and, for the last dim, the offsets themselves in a
// list beside it and the flags described in tm_internal.h in bits 28..29).
// The linear final coordinate of point q is then v(q) = sum_d C_d[q_d] and its
// owner is T[v(q)]: the chain is evaluated once per coordinate, not per point.
//
// Kernels: table build; processor map (streaming int32 writes); stencil counting
// (persistent, work queue over (candidate, row block) items, tables in LDS); bytes
// and selection; matmul tile bitmaps; redistribution counting.  All arithmetic is
// exact integer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tm_internal.h"
#include "tm_chain.h"

namespace tmk {

// ------------------------------------------------------------------ helpers

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t uniform32(int32_t x) {
    return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}

// Copies `words` int32 (a multiple of 4, both ends 16-byte aligned) from global
// memory to LDS with the workgroup's 256 threads: 16-byte loads, four in flight.
__device__ __forceinline__ void stage_words(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                            int32_t words) {
    const i32x4* s4 = reinterpret_cast<const i32x4*>(src);
    i32x4* d4 = reinterpret_cast<i32x4*>(dst);
    const int32_t n4 = words >> 2;
    int32_t i = threadIdx.x;
    for (; i + 3 * 256 < n4; i += 4 * 256) {
        const i32x4 a = s4[i], b = s4[i + 256], c = s4[i + 512], d = s4[i + 768];
        d4[i] = a;
        d4[i + 256] = b;
        d4[i + 512] = c;
        d4[i + 768] = d;
    }
    for (; i < n4; i += 256) d4[i] = s4[i];
}

// Sum over the wave of non-negative per-lane counts, in 64 bits (a wave's counts for
// one work item can exceed 2^31 on very long rows).
__device__ __forceinline__ unsigned long long wave_sum64(int v) {
    unsigned long long s = (unsigned long long)(unsigned)v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// ------------------------------------------------------------------ class-tuple counting

constexpr int kFoundCache = 4;  // distinct foreign owners held in registers per tuple


// Counts the class tuples t0, t0 + step, ... below tb of one candidate (tuples in C
// order over its per-dim classes, last dim fastest): per tuple the distinct foreign
// owners (and those on another node) of its cells, times its weight.
__device__ __forceinline__ void count_tuples(const int32_t* __restrict__ T, const int32_t* const (&CE)[TM_MAX_LRANK],
                                             const int32_t* const (&CS)[TM_MAX_LRANK],
                                             const int32_t* const (&CO)[TM_MAX_LRANK],
                                             const int32_t (&R)[TM_MAX_LRANK], int K, int gbits, int hs, int64_t tb,
                                             int64_t t0, int32_t step, unsigned long long& cnt,
                                             unsigned long long& icnt) {
    const int32_t RL = R[K - 1];
    // tuple t -> (row, k): row over the outer dims, k the last dim's class
    int64_t t = t0;
    int32_t row = (int32_t)(t / RL), k = (int32_t)(t - (int64_t)row * RL);
    const int32_t qs = step / RL, rs = step % RL;
    int32_t mrow = -1, vo = 0;
    int64_t wo = 1;
    // per outer dim of the current row: offset count and the offset list's position
    int32_t ndo[TM_MAX_LRANK], odo[TM_MAX_LRANK];
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) ndo[d] = odo[d] = 0;
    for (; t < tb; t += step) {
        if (row != mrow) {  // outer classes of this row: contribution, weight, offset lists
            uint32_t rr = (uint32_t)row;
            vo = 0;
            wo = 1;
#pragma unroll
            for (int d = TM_MAX_LRANK - 2; d >= 0; --d) {  // unrolled: the arrays stay in registers
                if (d > K - 2) continue;
                const uint32_t kd = rr % (uint32_t)R[d];
                rr /= (uint32_t)R[d];
                const int32_t e = CE[d][kd];
                vo += e & kValMask;
                ndo[d] = (e >> kCntShift) & 0xf;
                odo[d] = (int32_t)kd * hs;
                wo *= CS[d][kd + 1] - CS[d][kd];
            }
            mrow = row;
        }
        const int32_t el = CE[K - 1][k];
        const int32_t v = vo + (el & kValMask);
        const int64_t w = wo * (int64_t)(CS[K - 1][k + 1] - CS[K - 1][k]);
        const int32_t o = T[v];
        const int32_t onode = o >> gbits;
        int32_t f[kFoundCache];
        int nf = 0, c = 0, ic = 0;
#pragma unroll
        for (int d = 0; d < TM_MAX_LRANK; ++d) {
            if (d >= K) continue;
            const int32_t nd = d == K - 1 ? (el >> kCntShift) & 0xf : ndo[d];
            const int32_t* od = CO[d] + (d == K - 1 ? k * hs : odo[d]);
            for (int i = 0; i < nd; ++i) {
                const int32_t ot = T[v + od[i]];
                if (ot == o) continue;
                bool seen = false;
#pragma unroll
                for (int u = 0; u < kFoundCache; ++u) seen = seen || (u < nf && f[u] == ot);
                if (!seen && nf > kFoundCache) {
                    // more distinct owners than the cache holds: look at every earlier offset
                    for (int d2 = 0; d2 <= d && !seen; ++d2) {
                        const int32_t n2 = d2 == K - 1 ? (el >> kCntShift) & 0xf : ndo[d2];
                        const int32_t* o2 = CO[d2] + (d2 == K - 1 ? k * hs : odo[d2]);
                        const int e2 = d2 < d ? n2 : i;
                        for (int i2 = 0; i2 < e2 && !seen; ++i2) seen = T[v + o2[i2]] == ot;
                    }
                }
                if (seen) continue;
#pragma unroll
                for (int u = 0; u < kFoundCache; ++u) f[u] = u == nf ? ot : f[u];
                ++nf;
                ++c;
                ic += (ot >> gbits) != onode ? 1 : 0;
            }
        }
        cnt += (unsigned long long)w * (unsigned long long)c;
        icnt += (unsigned long long)w * (unsigned long long)ic;
        k += rs;
        row += qs;
        if (k >= RL) {
            k -= RL;
            ++row;
        }
    }
}

// ------------------------------------------------------------------ table build

// Sorted distinct non-zero offsets C[x +- s] - C[x] (1 <= s <= h, in-domain
// neighbours) of coordinate x, in slots o[0..n); unused slots hold INT32_MAX.
__device__ __forceinline__ int coord_offsets(const int32_t* __restrict__ C, int64_t x, int64_t l, int h,
                                             int32_t (&o)[2 * kMaxHalo]) {
#pragma unroll
    for (int i = 0; i < 2 * kMaxHalo; ++i) o[i] = INT32_MAX;
    const int32_t cv = C[x];
    int n = 0;
#pragma unroll
    for (int s = 1; s <= kMaxHalo; ++s) {
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
            const int64_t xx = dir ? x + s : x - s;
            if (s > h || xx < 0 || xx >= l) continue;
            const int32_t dv = C[xx] - cv;
            bool seen = dv == 0;
#pragma unroll
            for (int i = 0; i < 2 * kMaxHalo; ++i) seen = seen || o[i] == dv;
            if (seen) continue;
            // insert into the sorted slots (static indices only: no scratch)
#pragma unroll
            for (int i = 2 * kMaxHalo - 1; i >= 0; --i) {
                const bool shift = i > 0 && o[i - 1] > dv;
                const bool here = i == 0 ? o[0] > dv : (o[i - 1] <= dv && o[i] > dv);
                o[i] = shift ? o[i - 1] : (here ? dv : o[i]);
            }
            ++n;
        }
    }
    return n;
}

constexpr int kBuildStage = 2048;  // coordinate-table entries staged in LDS for the class build

// The owner table T[v] (one key per final-space coordinate), the coordinate tables
// C_d and, with halos (use_halo), the coordinate classes of every launch dim (see
// tm_internal.h): a coordinate starts a class when its contribution or offset set
// differs from its left neighbour's; class indices come from a workgroup prefix
// count of the starts.  With split, one workgroup per (candidate, launch dim) --
// workgroup d writes the d-th K-th of T, C_d and dim d's classes (small batches:
// more workgroups in flight) -- else one per candidate, all dims in turn (grid-
// stride in both cases).  The first workgroup of a candidate also writes its
// entries of the item table and, with out/counter, zeroes its outputs (workgroup 0
// of the launch the counting kernel's counters).
__global__ __launch_bounds__(256) void k_build_tables(const DevHeader* __restrict__ hdr,
                                                      const DevCand* __restrict__ cands,
                                                      int32_t* __restrict__ arena, int use_halo,
                                                      tm_stencil_cost* __restrict__ out,
                                                      unsigned long long* __restrict__ counter, int split) {
    __shared__ DevCand sc;
    __shared__ int32_t s_wt[4];
    __shared__ int32_t s_ct[kBuildStage];
    __shared__ float s_rt[kRecipSlots];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    const int upc = split ? TM_MAX_LRANK : 1;  // units per candidate
    const int64_t units = hdr->n * upc;
    if (counter && blockIdx.x == 0 && tid < 2) counter[tid] = 0ull;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t ci = u / upc;
        const int dlo = (int)(u - ci * upc);
        const int K = (int)__builtin_amdgcn_readfirstlane((uint32_t)cands[ci].lrank);
        if (dlo >= K) continue;  // uniform
        const int dhi = split ? dlo + 1 : K;
        lds_sync(nw);
        stage_cand(&sc, &cands[ci]);
        lds_sync(nw);
        op_reciprocals(sc, s_rt, tid, blockDim.x);
        lds_sync(nw);
        int32_t* base = arena + sc.arena_off;
        if (dlo == 0) {
            if (out && tid < 4) reinterpret_cast<int64_t*>(&out[ci])[tid] = 0;
            if (use_halo)  // this candidate's entries of the item table (work item -> candidate)
                for (int32_t j = tid; j < sc.citems; j += blockDim.x)
                    arena[hdr->item_tab + sc.item_first + j] = (int32_t)ci;
        }
        // node-level tables keep the node of each owner (GPU bits cleared): the
        // counting kernel then counts distinct other nodes per cell
        const int32_t keep = hdr->node_level ? ~((1 << sc.gbits) - 1) : -1;
        const int32_t v0 = split ? (int32_t)((int64_t)sc.vol * dlo / K) : 0;
        const int32_t v1 = split ? (int32_t)((int64_t)sc.vol * (dlo + 1) / K) : sc.vol;
        owner_keys_sized(sc, s_rt, base, 0, v0, v1, keep, tid, blockDim.x);
        for (int d = dlo; d < dhi; ++d) {
            if (d > dlo) lds_sync(nw);  // the previous dim's staged table is no longer read
            const int64_t l = sc.extent[d];
            int32_t* ct = base + sc.coord_off[d];
            // the dim's coordinate table; kept in LDS too when it fits (the class build
            // reads it 2 (2h + 1) times per coordinate)
            const bool staged = use_halo && l <= kBuildStage;
            for (int64_t x = tid; x < l; x += blockDim.x) {
                const int32_t cv = coord_value(sc, d, x);
                ct[x] = cv;
                if (staged) s_ct[x] = cv;
            }
            if (d == K - 1)  // zero entries up to a multiple of 512 (read in whole chunks)
                for (int64_t x = l + tid; x < ((l + 511) & ~int64_t(511)); x += blockDim.x) ct[x] = 0;
            if (!use_halo) continue;
            // the coordinate table complete (read from LDS when staged, else from global memory)
            if (staged) lds_sync(nw);
            else __syncthreads();
            const int32_t* cr = staged ? s_ct : ct;
            const int hs = sc.hstride;
            int32_t* rec = base + sc.cls_base;
            const int h = hdr->halo[d];
            const int64_t cap = sc.cls_cap[d];
            int32_t* ce = base + sc.cls_off[d];
            int32_t* cs = ce + ((cap + 3) & ~int64_t(3));
            int32_t* co = cs + ((cap + 4) & ~int64_t(3));
            int64_t run = 0;  // classes so far (the same in every thread)
            for (int64_t x0 = 0; x0 < l; x0 += blockDim.x) {
                const int64_t x = x0 + tid;
                bool start = false;
                int32_t val = 0, o[2 * kMaxHalo];
                int no = 0;
                if (x < l) {
                    val = cr[x];
                    no = coord_offsets(cr, x, l, h, o);
                    start = x == 0;
                    if (!start) {
                        int32_t pv[2 * kMaxHalo];
                        (void)coord_offsets(cr, x - 1, l, h, pv);
                        start = cr[x - 1] != val;
#pragma unroll
                        for (int i = 0; i < 2 * kMaxHalo; ++i) start = start || pv[i] != o[i];
                    }
                }
                const uint64_t m = __ballot(start);
                int64_t below = 0, tot = __popcll(m);
                if (nw > 1) {  // the other waves' starts (a one-wave workgroup has them all in m)
                    if (lane == 0) s_wt[wid] = __popcll(m);
                    __syncthreads();
                    tot = 0;
                    for (int w = 0; w < nw; ++w) {
                        below += w < wid ? s_wt[w] : 0;
                        tot += s_wt[w];
                    }
                }
                if (start) {
                    const int64_t idx = run + below + __builtin_amdgcn_mbcnt_hi(
                                                              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (idx < cap) {  // the capacity bounds the count (class_cap); never exceeded
                        ce[idx] = val | (no << kCntShift);
                        cs[idx] = (int32_t)x;
                        for (int i = 0; i < hs; ++i) co[idx * hs + i] = i < no ? o[i] : 0;
                    }
                }
                run += tot;
                if (nw > 1) __syncthreads();  // s_wt is rewritten by the next chunk
            }
            if (tid == 0) {
                if (run <= cap) cs[run] = (int32_t)l;
                rec[d] = run <= cap ? (int32_t)run : -1;  // -1: poisoned (counted as such)
            }
        }
    }
}

hipError_t launch_build_tables(const DevHeader* hdr, const DevCand* cands, int64_t n, int32_t* arena,
                               int32_t use_halo, hipStream_t s, tm_stencil_cost* out,
                               unsigned long long* counter) {
    // small batches: a workgroup per (candidate, launch dim); large ones: per candidate
    const int split = n <= kSplitBuildBatch ? 1 : 0;
    const int64_t units = n * (split ? TM_MAX_LRANK : 1);
    const int64_t grid = units < 131072 ? (units > 0 ? units : 1) : 131072;
    const int bs = n >= kSmallBlockBatch ? 64 : 256;
    hipLaunchKernelGGL(k_build_tables, dim3((unsigned)grid), dim3(bs), 0, s, hdr, cands, arena, use_halo, out,
                       counter, split);
    return hipGetLastError();
}

// ------------------------------------------------------------------ reset

__global__ void k_reset(DevHeader* hdr, unsigned long long* counter, tm_stencil_cost* out, int64_t cap) {
    const int64_t n = hdr->n < cap ? hdr->n : cap;
    int64_t* o = reinterpret_cast<int64_t*>(out);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 4 * n;
         i += (int64_t)gridDim.x * blockDim.x)
        o[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) counter[threadIdx.x] = 0ull;  // work and completion counters
}

hipError_t launch_reset(DevHeader* hdr, unsigned long long* counter, tm_stencil_cost* out, int64_t n,
                        hipStream_t s) {
    int64_t grid = (4 * n + 255) / 256;
    if (grid < 1) grid = 1;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_reset, dim3((unsigned)grid), dim3(256), 0, s, hdr, counter, out, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ stencil counting
//
// The distinct foreign owners of a cell depend only on the class of its coordinate
// along every launch dim (tm_internal.h): the cell's linear final index is the sum
// of the classes' contributions, and its star neighbours sit at that index plus
// the classes' offsets.  So a candidate's count is a sum over the tuples of its
// per-dim classes (the Cartesian product), each tuple evaluated once and weighted
// by the number of cells it stands for, the product of its classes' run lengths.
//
// A work item is a contiguous range of one candidate's class tuples in C order
// (last dim fastest); a candidate's items split its tuples evenly.  Workgroups take
// items from a global atomic counter (the next one is requested while the current
// one runs) and stage the candidate's owner table and class blocks in LDS when the
// candidate changes and they fit (else they are read from global memory).  Each
// thread evaluates every 256th tuple of the item: owner o = T[v], then the owners
// T[v + delta] over the classes' offsets; the distinct ones other than o are
// counted (and those on another node) times the tuple's weight, in 64 bits.  Waves
// reduce, and one 64-bit atomic per wave and item adds to the candidate's totals.


__device__ void finalize_select_block(const DevHeader* __restrict__ hdr, tm_stencil_cost* __restrict__ out,
                                      int64_t* __restrict__ best, int64_t* sb, int64_t* si, int64_t* sx);

__global__ __launch_bounds__(256) void k_count(const DevHeader* __restrict__ hdr, const DevCand* __restrict__ cands,
                                               const int32_t* __restrict__ arena,
                                               unsigned long long* __restrict__ counter,
                                               tm_stencil_cost* __restrict__ out, int fin,
                                               int64_t* __restrict__ best) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];
    __shared__ long long s_item;
    __shared__ int32_t s_cand;
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t total = uniform64(hdr->total_items);
    const int32_t budget = uniform32(hdr->cnt_words);  // LDS words of this launch

    int64_t cur = -1;
    int K = 1, gbits = 0, hs = 0, nit = 1;
    int64_t ifirst = 0;
    bool poisoned = false;
    int32_t R[TM_MAX_LRANK];
    const int32_t* T = arena;
    const int32_t* CE[TM_MAX_LRANK];
    const int32_t* CS[TM_MAX_LRANK];
    const int32_t* CO[TM_MAX_LRANK];
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) {
        R[d] = 1;
        CE[d] = CS[d] = CO[d] = arena;
    }

    // workgroup b takes item b first; the later items come from the work counter
    // (items gridDim.x, gridDim.x + 1, ...), the next one and its candidate (from the
    // item table) fetched while the current item runs
    const int32_t* __restrict__ itab = arena + hdr->item_tab;
    unsigned long long next = blockIdx.x;
    int32_t next_c = 0;
    if (tid == 0) next_c = (int64_t)next < total ? itab[next] : 0;
    for (;;) {
        if (tid == 0) {
            s_item = (long long)next;
            s_cand = next_c;
        }
        __syncthreads();
        const int64_t item = uniform64(s_item);
        const int64_t lo = uniform32(s_cand);
        __syncthreads();
        if (item >= total) break;
        if (tid == 0) {
            next = gridDim.x + atomicAdd(counter, 1ull);
            next_c = (int64_t)next < total ? itab[next] : 0;
        }
        if (lo != cur) {
            const DevCand* c = &cands[lo];
            const int32_t* src = arena + c->arena_off;
            const int32_t vol = uniform32(c->vol), cb = uniform32(c->cls_base), cw = uniform32(c->cls_words);
            const int32_t tw = (vol + 3) & ~3;
            const bool staged = tw + cw <= budget;
            __syncthreads();  // the previous candidate's staged tables are no longer read
            if (staged) {  // both regions 16-byte aligned, whole multiples of 4 words
                stage_words(lds, src, tw);
                stage_words(lds + tw, src + cb, cw);
            }
            T = staged ? lds : src;
            K = uniform32(c->lrank);
            gbits = uniform32(c->gbits);
            hs = uniform32(c->hstride);
            nit = uniform32(c->citems);
            ifirst = uniform64(c->item_first);
            poisoned = false;
#pragma unroll
            for (int d = 0; d < TM_MAX_LRANK; ++d) {
                R[d] = 1;
                if (d < K) {
                    R[d] = uniform32(src[cb + d]);
                    poisoned = poisoned || R[d] < 0;
                    const int64_t cap = uniform32(c->cls_cap[d]);
                    const int32_t rel = uniform32(c->cls_off[d]);  // dim d's block, from the arena or LDS
                    CE[d] = staged ? lds + tw + (rel - cb) : src + rel;
                    CS[d] = CE[d] + ((cap + 3) & ~int64_t(3));
                    CO[d] = CS[d] + ((cap + 4) & ~int64_t(3));
                }
            }
            cur = lo;
            __syncthreads();
        }
        if (poisoned) {  // a class block overflowed its capacity: make the result unmistakable
            if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].ghost_cells), 1ull << 62);
            continue;
        }
        // this item's tuples [ta, tb) of the candidate's N = prod R_d, split evenly
        const int64_t j = item - ifirst;
        int64_t N = 1;
        for (int d = 0; d < K; ++d) N *= R[d];
        const int64_t q = N / nit, r = N % nit;
        const int64_t ta = j * q + (j < r ? j : r);
        const int64_t tb = ta + q + (j < r ? 1 : 0);
        unsigned long long cnt = 0, icnt = 0;
        count_tuples(T, CE, CS, CO, R, K, gbits, hs, tb, ta + tid, 256, cnt, icnt);
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            cnt += __shfl_xor(cnt, o2, 64);
            icnt += __shfl_xor(icnt, o2, 64);
        }
        if (lane == 0 && (cnt | icnt)) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].ghost_cells), cnt);
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].inter_cells), icnt);
        }
    }
    if (!fin) return;
    // the last workgroup to finish writes the bytes and selects
    __shared__ int64_t sb[256], si[256], sx[256];
    __syncthreads();
    if (tid == 0) {
        __threadfence();  // this workgroup's counts are visible before it reports done
        s_last = atomicAdd(counter + 1, 1ull) == (unsigned long long)gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finalize_select_block(hdr, out, best, sb, si, sx);
}

int count_kernel_occupancy(int lds_words, int* blocks_per_cu) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_count), 256,
                                                     (size_t)lds_words * 4) != hipSuccess)
        return -1;
    *blocks_per_cu = nb;
    return 0;
}

hipError_t launch_count(const DevHeader* hdr, const DevCand* cands, const int32_t* arena,
                        unsigned long long* counter, tm_stencil_cost* out, int grid, int lds_words,
                        hipStream_t s, bool fin, int64_t* best) {
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(256), (size_t)lds_words * 4, s, hdr, cands, arena, counter, out,
                       fin ? 1 : 0, best);
    return hipGetLastError();
}

// Sum over candidates of the product of their class counts (the counting work).
__global__ __launch_bounds__(256) void k_class_tuples(const DevCand* __restrict__ cands, int64_t n,
                                                      const int32_t* __restrict__ arena,
                                                      unsigned long long* __restrict__ total) {
    unsigned long long acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const DevCand& c = cands[i];
        const int32_t* rec = arena + c.arena_off + c.cls_base;
        unsigned long long t = 1;
        for (int d = 0; d < c.lrank; ++d) t *= (unsigned long long)(rec[d] > 0 ? rec[d] : 0);
        acc += t;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(total, acc);
}

hipError_t launch_class_tuples(const DevCand* cands, int64_t n, const int32_t* arena, unsigned long long* total,
                               hipStream_t s) {
    const int64_t grid = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(k_class_tuples, dim3((unsigned)grid), dim3(256), 0, s, cands, n, arena, total);
    return hipGetLastError();
}

// ------------------------------------------------------------------ bytes + selection

// One workgroup: bytes from cell counts, then the minimum of (bytes, inter_bytes,
// index) -> *best (when given).  The counts are read at device scope (the counting
// kernel's atomics).
__device__ void finalize_select_block(const DevHeader* __restrict__ hdr, tm_stencil_cost* __restrict__ out,
                                      int64_t* __restrict__ best, int64_t* sb, int64_t* si, int64_t* sx) {
    const int nt = blockDim.x, t = threadIdx.x;
    const int64_t n = hdr->n;
    const int64_t eb = hdr->elem_bytes;
    int64_t kb = INT64_MAX, ki = INT64_MAX, kx = INT64_MAX;
    for (int64_t i = t; i < n; i += nt) {
        int64_t* o = reinterpret_cast<int64_t*>(&out[i]);
        const int64_t gc = __hip_atomic_load(o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t ic = __hip_atomic_load(o + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t b = gc * eb, ib = ic * eb;
        o[2] = b;
        o[3] = ib;
        if (b < kb || (b == kb && (ib < ki || (ib == ki && i < kx)))) {
            kb = b;
            ki = ib;
            kx = i;
        }
    }
    sb[t] = kb;
    si[t] = ki;
    sx[t] = kx;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (t < w) {
            const int o = t + w;
            if (sb[o] < sb[t] || (sb[o] == sb[t] && (si[o] < si[t] || (si[o] == si[t] && sx[o] < sx[t])))) {
                sb[t] = sb[o];
                si[t] = si[o];
                sx[t] = sx[o];
            }
        }
        __syncthreads();
    }
    if (t == 0 && best) *best = n > 0 ? sx[0] : -1;
}

__global__ __launch_bounds__(1024) void k_finalize_select(const DevHeader* __restrict__ hdr,
                                                          tm_stencil_cost* __restrict__ out,
                                                          int64_t* __restrict__ best) {
    __shared__ int64_t sb[1024], si[1024], sx[1024];
    finalize_select_block(hdr, out, best, sb, si, sx);
}

// Bytes from cell counts only (no selection), grid-stride over the candidates.
__global__ __launch_bounds__(256) void k_finalize_bytes(const DevHeader* __restrict__ hdr,
                                                        tm_stencil_cost* __restrict__ out) {
    const int64_t n = hdr->n, eb = hdr->elem_bytes;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t* o = reinterpret_cast<int64_t*>(&out[i]);
        const int64_t gc = __hip_atomic_load(o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t ic = __hip_atomic_load(o + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        o[2] = gc * eb;
        o[3] = ic * eb;
    }
}

hipError_t launch_finalize_select(const DevHeader* hdr, tm_stencil_cost* out, int64_t* best, int64_t n_max,
                                  hipStream_t s) {
    if (!best && n_max > kFinBytesGrid) {
        const int64_t g = std::min<int64_t>((n_max + 255) / 256, 2048);
        hipLaunchKernelGGL(k_finalize_bytes, dim3((unsigned)g), dim3(256), 0, s, hdr, out);
    } else {
        hipLaunchKernelGGL(k_finalize_select, dim3(1), dim3(1024), 0, s, hdr, out, best);
    }
    return hipGetLastError();
}

// One workgroup per segment.
// Ties on (bytes, inter_bytes) go to the smallest tie key: key[i] when given (the
// original candidate index of a gathered sub-batch), else i.  Writes the position.
__global__ __launch_bounds__(256) void k_select_segments(const tm_stencil_cost* __restrict__ costs,
                                                         const int64_t* __restrict__ seg,
                                                         const int64_t* __restrict__ key,
                                                         int64_t* __restrict__ best) {
    __shared__ int64_t sb[256], si[256], sx[256], sp[256];
    const int64_t a = seg[blockIdx.x], e = seg[blockIdx.x + 1];
    int64_t kb = INT64_MAX, ki = INT64_MAX, kx = INT64_MAX, kp = INT64_MAX;
    for (int64_t i = a + threadIdx.x; i < e; i += blockDim.x) {
        const int64_t b = costs[i].bytes, ib = costs[i].inter_bytes;
        const int64_t x = key ? key[i] : i;
        if (b < kb || (b == kb && (ib < ki || (ib == ki && x < kx)))) {
            kb = b;
            ki = ib;
            kx = x;
            kp = i;
        }
    }
    sp[threadIdx.x] = kp;
    sb[threadIdx.x] = kb;
    si[threadIdx.x] = ki;
    sx[threadIdx.x] = kx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (sb[o] < sb[threadIdx.x] ||
                (sb[o] == sb[threadIdx.x] &&
                 (si[o] < si[threadIdx.x] || (si[o] == si[threadIdx.x] && sx[o] < sx[threadIdx.x])))) {
                sb[threadIdx.x] = sb[o];
                si[threadIdx.x] = si[o];
                sx[threadIdx.x] = sx[o];
                sp[threadIdx.x] = sp[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) best[blockIdx.x] = e > a ? sp[0] - a : -1;
}

hipError_t launch_select_segments(const tm_stencil_cost* costs, const int64_t* seg, int64_t nseg,
                                  int64_t* best, hipStream_t s, const int64_t* key) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select_segments, dim3((unsigned)nseg), dim3(256), 0, s, costs, seg, key, best);
    return hipGetLastError();
}

// ------------------------------------------------------------------ processor map
//
// Each workgroup writes contiguous blocks of map_rows_per_block(L) rows (about 2,048
// points, 8 KB), its 256 threads stepping through the block's 16-byte pieces in
// order (one 16-byte store per thread and step when rows start 16-byte aligned, else
// one point).  The owner table and (when it fits) the last dim's coordinate table
// sit in LDS, and so do the block's row bases (sums of the outer dims' entries).
// Measured on a 512^3 map: 8 KB blocks with plain stores
// 6.80 TB/s, 16 KB 6.05, 4 KB 5.71, non-temporal stores 5.75 at 16 KB; a plain
// device fill of the same bytes 6.58.

template <int NT>
__global__ __launch_bounds__(NT) void k_map(const DevCand* __restrict__ cands, int64_t n,
                                            const int32_t* __restrict__ arena,
                                            const int64_t* __restrict__ d_index, int64_t index,
                                            int32_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // 16-byte aligned: ds_read_b128 of staged tables
    // a short prologue (many small workgroups): the descriptor's fields are read in
    // place; the tables and the first block's row bases are ready behind one barrier
    __shared__ int32_t s_base[kMapMaxRowsPerBlock];
    static_assert(NT >= kMapMaxRowsPerBlock, "a thread per row base");
    const int64_t ci = d_index ? uniform64(*d_index) : index;
    if (ci < 0 || ci >= n) return;  // no candidate selected (empty batch)
    const DevCand* __restrict__ c = &cands[ci];
    const int32_t words = uniform32(c->lds_words);
    const int32_t* G = arena + uniform64(c->arena_off);  // outer tables (and a last-dim table that did not fit)
    {
        const i32x4* s4 = reinterpret_cast<const i32x4*>(G);
        i32x4* d4 = reinterpret_cast<i32x4*>(lds);
        for (int32_t i = threadIdx.x; i < (words + 3) >> 2; i += NT) d4[i] = s4[i];
    }
    const int K = uniform32(c->lrank);
    const int32_t L = uniform32(c->L);
    const int64_t rows = uniform64(c->rows);
    const int32_t gb = uniform32(c->gbits), g = uniform32(c->gpus), gmask = (1 << gb) - 1;
    const int32_t* CL = uniform32(c->cl_lds) ? lds + uniform32(c->coord_off[K - 1]) : G + uniform32(c->coord_off[K - 1]);
    int32_t co[TM_MAX_LRANK];
    uint32_t ex[TM_MAX_LRANK];
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) {
        co[d] = d < K - 1 ? uniform32(c->coord_off[d]) : 0;
        ex[d] = d < K - 1 ? (uint32_t)uniform64(c->extent[d]) : 1u;
    }
    const int32_t* T = lds;
    const int tid = threadIdx.x;
    const int32_t rpb = map_rows_per_block(L, NT == 64);
    const bool vec = (L & 3) == 0 && ((reinterpret_cast<uintptr_t>(out) & 15) == 0);
    const int64_t stride = (int64_t)gridDim.x * rpb;
    for (int64_t r0 = (int64_t)blockIdx.x * rpb; r0 < rows; r0 += stride) {
        const int32_t nr = (int32_t)(rows - r0 < rpb ? rows - r0 : rpb);
        // the block's row bases: the sums of the outer dims' entries of its rows
        if (tid < nr) {
            uint32_t rr = (uint32_t)(r0 + tid);
            int32_t bl = 0;
            for (int d = K - 2; d >= 0; --d) {
                bl += G[co[d] + (int32_t)(rr % ex[d])] & kValMask;
                rr /= ex[d];
            }
            s_base[tid] = bl;
        }
        __syncthreads();  // tables (first block) and bases ready
        int32_t* blk = out + r0 * (int64_t)L;
        if (vec) {
            const uint32_t pr = (uint32_t)L >> 2;  // 16-byte pieces per row
            const uint32_t np = (uint32_t)nr * pr;
            for (uint32_t j = tid; j < np; j += NT) {
                const uint32_t rl = j / pr;
                const int32_t x = (int32_t)(j - rl * pr) * 4;
                const int32_t base = s_base[rl];
                i32x4 key;
                key.x = T[base + (CL[x] & kValMask)];
                key.y = T[base + (CL[x + 1] & kValMask)];
                key.z = T[base + (CL[x + 2] & kValMask)];
                key.w = T[base + (CL[x + 3] & kValMask)];
                reinterpret_cast<i32x4*>(blk)[j] = (key >> gb) * g + (key & gmask);
            }
        } else {
            const uint32_t np = (uint32_t)nr * (uint32_t)L;
            for (uint32_t j = tid; j < np; j += NT) {
                const uint32_t rl = j / (uint32_t)L;
                const int32_t x = (int32_t)(j - rl * (uint32_t)L);
                const int32_t key = T[s_base[rl] + (CL[x] & kValMask)];
                blk[j] = (key >> gb) * g + (key & gmask);
            }
        }
        if (r0 + stride < rows) __syncthreads();  // the next block rewrites the bases
    }
}

hipError_t launch_map(const DevCand* cands, int64_t n, const int32_t* arena, const int64_t* d_index,
                      int64_t index, int32_t* out, int grid, int lds_words, hipStream_t s) {
    if (map_narrow(lds_words))
        hipLaunchKernelGGL(k_map<64>, dim3(grid), dim3(64), (size_t)lds_words * 4, s, cands, n, arena, d_index,
                           index, out);
    else
        hipLaunchKernelGGL(k_map<256>, dim3(grid), dim3(256), (size_t)lds_words * 4, s, cands, n, arena, d_index,
                           index, out);
    return hipGetLastError();
}

// Chain table as processor ids (for inspection and tests).
__global__ void k_chain_table(const DevCand* __restrict__ cand, const int32_t* __restrict__ arena,
                              int32_t* __restrict__ out) {
    const DevCand& c = *cand;
    const int32_t gmask = (1 << c.gbits) - 1;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < c.vol; v += gridDim.x * blockDim.x) {
        const int32_t key = arena[c.arena_off + v];
        out[v] = (key >> c.gbits) * c.gpus + (key & gmask);
    }
}

hipError_t launch_chain_table(const DevCand* cand, const int32_t* arena, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_chain_table, dim3(256), dim3(256), 0, s, cand, arena, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ redistribution
//
// Pairs (a, b) of mappings of one launch domain: candidates [0, npair) of the batch
// are the a's, [npair, 2 npair) the b's.  A cell moves when its owner under a
// differs from its owner under b, and both owners are fixed by the pair of its
// coordinate's contributions along every launch dim: consecutive coordinates with
// the same pair (C^a_d[x], C^b_d[x]) form a joint class, and the moved cells are a
// sum over tuples of joint classes, one owner comparison per tuple weighted by the
// cells it stands for (exactly the per-cell count, regrouped).  k_pair_classes
// builds each pair's joint classes (one workgroup per pair, a workgroup prefix count
// of class starts), writes the item table and zeroes the pair's outputs; k_pair_count
// takes (pair, tuple range) items from a work queue, as the stencil counting does.
// The pair's class block sits in a's table block (cls_base, cls_off, cls_cap of the
// a-side descriptor): record of the class counts, then per dim the a entries, the b
// entries and the run starts of its classes.

__global__ __launch_bounds__(256) void k_pair_classes(const DevCand* __restrict__ cands, int64_t npair,
                                                      int32_t* __restrict__ arena, int64_t item_tab,
                                                      tm_redist_cost* __restrict__ out,
                                                      unsigned long long* __restrict__ counter) {
    __shared__ int32_t s_wt[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (blockIdx.x == 0 && tid < 2) counter[tid] = 0ull;
    for (int64_t i = blockIdx.x; i < npair; i += gridDim.x) {
        const DevCand* __restrict__ a = &cands[i];
        const DevCand* __restrict__ b = &cands[npair + i];
        const int K = uniform32(a->lrank);
        int32_t* A = arena + uniform64(a->arena_off);
        const int32_t* B = arena + uniform64(b->arena_off);
        if (tid < 4) reinterpret_cast<int64_t*>(&out[i])[tid] = 0;
        const int32_t nit = uniform32(a->citems);
        const int64_t first = uniform64(a->item_first);
        for (int32_t j = tid; j < nit; j += blockDim.x) arena[item_tab + first + j] = (int32_t)i;
        int32_t* rec = A + uniform32(a->cls_base);
        for (int d = 0; d < K; ++d) {
            const int64_t l = uniform64(a->extent[d]);
            const int32_t* ca = A + uniform32(a->coord_off[d]);
            const int32_t* cb = B + uniform32(b->coord_off[d]);
            const int64_t cap = uniform32(a->cls_cap[d]);
            int32_t* ea = A + uniform32(a->cls_off[d]);
            int32_t* eb = ea + ((cap + 3) & ~int64_t(3));
            int32_t* cs = eb + ((cap + 3) & ~int64_t(3));
            int64_t run = 0;  // classes so far (the same in every thread)
            for (int64_t x0 = 0; x0 < l; x0 += blockDim.x) {
                const int64_t x = x0 + tid;
                int32_t va = 0, vb = 0;
                bool start = false;
                if (x < l) {
                    va = ca[x] & kValMask;
                    vb = cb[x] & kValMask;
                    start = x == 0 || (ca[x - 1] & kValMask) != va || (cb[x - 1] & kValMask) != vb;
                }
                const uint64_t m = __ballot(start);
                if (lane == 0) s_wt[wid] = __popcll(m);
                __syncthreads();
                int64_t below = 0, tot = 0;
                for (int w = 0; w < 4; ++w) {
                    below += w < wid ? s_wt[w] : 0;
                    tot += s_wt[w];
                }
                if (start) {
                    const int64_t idx =
                        run + below + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (idx < cap) {  // the capacity bounds the count; never exceeded
                        ea[idx] = va;
                        eb[idx] = vb;
                        cs[idx] = (int32_t)x;
                    }
                }
                run += tot;
                __syncthreads();  // s_wt is rewritten by the next chunk
            }
            if (tid == 0) {
                if (run <= cap) cs[run] = (int32_t)l;
                rec[d] = run <= cap ? (int32_t)run : -1;  // -1: poisoned (counted as such)
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_pair_count(const DevCand* __restrict__ cands, int64_t npair,
                                                    const int32_t* __restrict__ arena, int64_t item_tab,
                                                    int64_t total, int32_t budget,
                                                    unsigned long long* __restrict__ counter,
                                                    tm_redist_cost* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];
    __shared__ long long s_item;
    __shared__ int32_t s_pair;
    const int tid = threadIdx.x, lane = tid & 63;
    const int32_t* __restrict__ itab = arena + item_tab;
    int64_t cur = -1;
    int K = 1, gbits = 0, nit = 1;
    int64_t ifirst = 0;
    bool poisoned = false;
    int32_t R[TM_MAX_LRANK];
    const int32_t* TA = arena;
    const int32_t* TB = arena;
    const int32_t* EA[TM_MAX_LRANK];
    const int32_t* EB[TM_MAX_LRANK];
    const int32_t* CS[TM_MAX_LRANK];
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) {
        R[d] = 1;
        EA[d] = EB[d] = CS[d] = arena;
    }
    // workgroup b takes item b first, the later ones from the work counter
    unsigned long long next = blockIdx.x;
    int32_t next_p = 0;
    if (tid == 0) next_p = (int64_t)next < total ? itab[next] : 0;
    for (;;) {
        if (tid == 0) {
            s_item = (long long)next;
            s_pair = next_p;
        }
        __syncthreads();
        const int64_t item = uniform64(s_item);
        const int64_t pi = uniform32(s_pair);
        __syncthreads();
        if (item >= total) break;
        if (tid == 0) {
            next = gridDim.x + atomicAdd(counter, 1ull);
            next_p = (int64_t)next < total ? itab[next] : 0;
        }
        if (pi != cur) {
            const DevCand* a = &cands[pi];
            const DevCand* b = &cands[npair + pi];
            const int32_t* A = arena + uniform64(a->arena_off);
            const int32_t* B = arena + uniform64(b->arena_off);
            const int32_t va = uniform32(a->vol), vb = uniform32(b->vol);
            const int32_t cbase = uniform32(a->cls_base), cw = uniform32(a->cls_words);
            const int32_t ta = (va + 3) & ~3, tb = (vb + 3) & ~3;
            const bool staged = ta + tb + cw <= budget;
            __syncthreads();  // the previous pair's staged tables are no longer read
            if (staged) {  // 16-byte aligned regions, whole multiples of 4 words
                stage_words(lds, A, ta);
                stage_words(lds + ta, B, tb);
                stage_words(lds + ta + tb, A + cbase, cw);
            }
            TA = staged ? lds : A;
            TB = staged ? lds + ta : B;
            K = uniform32(a->lrank);
            gbits = uniform32(a->gbits);
            nit = uniform32(a->citems);
            ifirst = uniform64(a->item_first);
            poisoned = false;
#pragma unroll
            for (int d = 0; d < TM_MAX_LRANK; ++d) {
                R[d] = 1;
                if (d < K) {
                    R[d] = uniform32(A[cbase + d]);
                    poisoned = poisoned || R[d] < 0;
                    const int64_t cap = uniform32(a->cls_cap[d]);
                    const int32_t rel = uniform32(a->cls_off[d]);
                    EA[d] = staged ? lds + ta + tb + (rel - cbase) : A + rel;
                    EB[d] = EA[d] + ((cap + 3) & ~int64_t(3));
                    CS[d] = EB[d] + ((cap + 3) & ~int64_t(3));
                }
            }
            cur = pi;
            __syncthreads();
        }
        if (poisoned) {  // a class block overflowed its capacity: make the result unmistakable
            if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].moved_cells), 1ull << 62);
            continue;
        }
        // this item's tuples [t0, t1) of the pair's N = prod R_d, split evenly
        const int64_t j = item - ifirst;
        int64_t N = 1;
        for (int d = 0; d < K; ++d) N *= R[d];
        const int64_t q = N / nit, r = N % nit;
        const int64_t t0 = j * q + (j < r ? j : r);
        const int64_t t1 = t0 + q + (j < r ? 1 : 0);
        const int32_t RL = R[K - 1];
        int64_t t = t0 + tid;
        int32_t row = (int32_t)(t / RL), k = (int32_t)(t - (int64_t)row * RL);
        const int32_t qs = 256 / RL, rs = 256 % RL;
        int32_t mrow = -1, ao = 0, bo = 0;
        int64_t wo = 1;
        unsigned long long mv = 0, iv = 0;
        for (; t < t1; t += 256) {
            if (row != mrow) {  // outer classes of this row: both contributions and the weight
                uint32_t rr = (uint32_t)row;
                ao = 0;
                bo = 0;
                wo = 1;
#pragma unroll
                for (int d = TM_MAX_LRANK - 2; d >= 0; --d) {
                    if (d > K - 2) continue;
                    const uint32_t kd = rr % (uint32_t)R[d];
                    rr /= (uint32_t)R[d];
                    ao += EA[d][kd];
                    bo += EB[d][kd];
                    wo *= CS[d][kd + 1] - CS[d][kd];
                }
                mrow = row;
            }
            const int32_t oa = TA[ao + EA[K - 1][k]], ob = TB[bo + EB[K - 1][k]];
            const int64_t w = wo * (int64_t)(CS[K - 1][k + 1] - CS[K - 1][k]);
            mv += oa != ob ? (unsigned long long)w : 0ull;
            iv += (oa >> gbits) != (ob >> gbits) ? (unsigned long long)w : 0ull;
            k += rs;
            row += qs;
            if (k >= RL) {
                k -= RL;
                ++row;
            }
        }
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            mv += __shfl_xor(mv, o2, 64);
            iv += __shfl_xor(iv, o2, 64);
        }
        if (lane == 0 && (mv | iv)) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].moved_cells), mv);
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].inter_cells), iv);
        }
    }
}

__global__ void k_redist_bytes(tm_redist_cost* __restrict__ out, int64_t npair, int64_t elem_bytes) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npair; i += (int64_t)gridDim.x * blockDim.x) {
        out[i].bytes = out[i].moved_cells * elem_bytes;
        out[i].inter_bytes = out[i].inter_cells * elem_bytes;
    }
}

hipError_t launch_redist(const DevCand* cands, int64_t npair, int32_t* arena, int64_t item_tab, int64_t items,
                         int64_t elem_bytes, tm_redist_cost* out, unsigned long long* counter, int grid,
                         int lds_words, hipStream_t s) {
    const int64_t pg = npair < 65536 ? (npair > 0 ? npair : 1) : 65536;
    hipLaunchKernelGGL(k_pair_classes, dim3((unsigned)pg), dim3(256), 0, s, cands, npair, arena, item_tab, out, counter);
    hipLaunchKernelGGL(k_pair_count, dim3(grid), dim3(256), (size_t)lds_words * 4, s, cands, npair,
                       (const int32_t*)arena, item_tab, items, lds_words, counter, out);
    const int zg = (int)std::min<int64_t>((npair + 255) / 256 + 1, 1024);
    hipLaunchKernelGGL(k_redist_bytes, dim3(zg), dim3(256), 0, s, out, npair, elem_bytes);
    return hipGetLastError();
}

// ------------------------------------------------------------------ matmul tiles
//
// A tile of A (i, k) is fetched by every processor that owns some task (i, j, k),
// and the owners along j depend only on the classes of i and k (runs of coordinates
// with the same contribution to the final index, built by the table build with a
// zero halo): all tiles of one pair of classes have the same owner set, and each
// processor of it counts the pair's tiles, the product of the two run lengths.  The
// same holds for B (k, j) over i and C (i, j) over k.  Work block = (candidate,
// matrix m in {A, B, C}, kMatmulTiles class pairs of the candidate's bound); a
// thread takes one class pair per step and walks the classes of the reduction dim,
// OR-ing each owner's bit into a bitmap of W 64-bit words in registers, then adds
// the pair's weight to every processor of its bitmap in LDS; the block's LDS counts
// go to the per-processor totals with one atomic per processor.

template <int W>
__global__ __launch_bounds__(256) void k_matmul(const DevCand* __restrict__ cands, int64_t n,
                                                const int32_t* __restrict__ arena,
                                                const int64_t* __restrict__ proc_off,
                                                unsigned long long* __restrict__ per_proc,
                                                const int64_t* __restrict__ block_first, int64_t total_blocks,
                                                int32_t budget) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // owner table and class blocks
    __shared__ unsigned long long s_cnt[64 * W];
    const int tid = threadIdx.x;
    int64_t cur = -1;
    const int32_t* T = arena;
    const int32_t* E[3];
    const int32_t* S[3];
    int32_t R[3] = {1, 1, 1};
    int32_t gb = 0, g = 1, P = 1;
    for (int i = tid; i < 64 * W; i += 256) s_cnt[i] = 0;
    for (int64_t blk = blockIdx.x; blk < total_blocks; blk += gridDim.x) {
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (block_first[mid] <= blk) lo = mid;
            else hi = mid - 1;
        }
        lo = uniform64(lo);
        if (lo != cur) {
            const DevCand* c = &cands[lo];
            const int32_t* src = arena + uniform64(c->arena_off);
            const int32_t vol = uniform32(c->vol), cb = uniform32(c->cls_base), cw = uniform32(c->cls_words);
            const int32_t tw = (vol + 3) & ~3;
            const bool staged = tw + cw <= budget;
            __syncthreads();  // the previous candidate's tables are no longer read
            if (staged) {
                stage_words(lds, src, tw);
                stage_words(lds + tw, src + cb, cw);
            }
            T = staged ? lds : src;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                R[d] = uniform32(src[cb + d]);
                const int64_t cap = uniform32(c->cls_cap[d]);
                const int32_t rel = uniform32(c->cls_off[d]);
                E[d] = staged ? lds + tw + (rel - cb) : src + rel;
                S[d] = E[d] + ((cap + 3) & ~int64_t(3));
            }
            gb = uniform32(c->gbits);
            g = uniform32(c->gpus);
            P = uniform32(c->nodes) * g;
            cur = lo;
            __syncthreads();
        }
        const int64_t b0 = block_first[lo];
        const int64_t c0 = uniform32(cands[lo].cls_cap[0]), c1 = uniform32(cands[lo].cls_cap[1]),
                      c2 = uniform32(cands[lo].cls_cap[2]);
        const int64_t bA = matmul_pair_blocks(c0, c2), bB = matmul_pair_blocks(c2, c1);
        int64_t local = blk - b0;
        int m;
        if (local < bA) m = 0;
        else if (local < bA + bB) { m = 1; local -= bA; }
        else { m = 2; local -= bA + bB; }
        // the matrix's fixed dims (a, b: tile = ca * R_b + cb) and reduction dim r:
        // A = (0, 2; 1), B = (2, 1; 0), C = (0, 1; 2), picked by selects (static indices)
        const bool mA = m == 0, mB = m == 1;
        const int32_t Ra = mB ? R[2] : R[0], Rb = mA ? R[2] : R[1], Rr = mA ? R[1] : (mB ? R[0] : R[2]);
        const int32_t* Ea = mB ? E[2] : E[0];
        const int32_t* Sa = mB ? S[2] : S[0];
        const int32_t* Eb = mA ? E[2] : E[1];
        const int32_t* Sb = mA ? S[2] : S[1];
        const int32_t* Er = mA ? E[1] : (mB ? E[0] : E[2]);
        unsigned long long* dst = per_proc + proc_off[lo] * 3;
        if (Ra < 0 || Rb < 0 || Rr < 0) {  // over capacity (never: the capacity bounds the count): poison
            if (tid == 0) atomicAdd(&dst[m], 1ull << 62);
            continue;
        }
        // t < Ra * Rb <= 2^31 (tile count of a matrix, checked by the host)
        const uint32_t ntile = (uint32_t)Ra * (uint32_t)Rb, t1 = (uint32_t)(local + 1) * kMatmulTiles;
        for (uint32_t t = (uint32_t)local * kMatmulTiles + tid; t < t1 && t < ntile; t += 256) {
            const int32_t ca = (int32_t)(t / (uint32_t)Rb), cbx = (int32_t)(t - (uint32_t)ca * (uint32_t)Rb);
            const int32_t fixed = (Ea[ca] & kValMask) + (Eb[cbx] & kValMask);
            const unsigned long long w =
                (unsigned long long)(Sa[ca + 1] - Sa[ca]) * (unsigned long long)(Sb[cbx + 1] - Sb[cbx]);
            uint64_t bm[W];
#pragma unroll
            for (int u = 0; u < W; ++u) bm[u] = 0;
            for (int32_t r = 0; r < Rr; ++r) {
                const int32_t key = T[fixed + (Er[r] & kValMask)];
                const int32_t p = (key >> gb) * g + (key & ((1 << gb) - 1));
                const uint64_t bit = 1ull << (p & 63);
                if (W == 1) {
                    bm[0] |= bit;
                } else {
#pragma unroll
                    for (int u = 0; u < W; ++u) bm[u] |= ((p >> 6) == u) ? bit : 0ull;
                }
            }
#pragma unroll
            for (int u = 0; u < W; ++u) {
                uint64_t b = bm[u];
                while (b) {
                    const int q = __builtin_ctzll(b);
                    b &= b - 1;
                    atomicAdd(&s_cnt[u * 64 + q], w);
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < 64 * W; i += 256) {
            const unsigned long long v = s_cnt[i];
            if (v) {
                if (i < P) atomicAdd(&dst[i * 3 + m], v);
                s_cnt[i] = 0;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_matmul(const DevCand* cands, int64_t n, const int32_t* arena, int words_max, int pmax,
                         const int64_t* proc_off, unsigned long long* per_proc, int64_t total_blocks,
                         const int64_t* block_first, hipStream_t s) {
    const int W = (pmax + 63) / 64;
    int64_t grid = total_blocks < 8192 ? total_blocks : 8192;
    if (grid < 1) grid = 1;
    const size_t lds = (size_t)words_max * 4;
#define TM_MM(w)                                                                                        \
    if (W <= w) {                                                                                       \
        hipLaunchKernelGGL(k_matmul<w>, dim3((unsigned)grid), dim3(256), lds, s, cands, n, arena, proc_off, \
                           per_proc, block_first, total_blocks, words_max);                             \
        return hipGetLastError();                                                                       \
    }
    TM_MM(1) TM_MM(2) TM_MM(4) TM_MM(8) TM_MM(16)
#undef TM_MM
    return hipErrorInvalidValue;
}

// Totals, maxima and bytes per candidate; optional copy of the per-processor counts.
__global__ __launch_bounds__(256) void k_matmul_finalize(const DevCand* __restrict__ cands,
                                                         const int64_t* __restrict__ proc_off,
                                                         const unsigned long long* __restrict__ per_proc,
                                                         int64_t tile_bytes, tm_matmul_cost* __restrict__ out,
                                                         int64_t* __restrict__ out_per_proc) {
    __shared__ unsigned long long st[3][256], sm[3][256];
    const int64_t c = blockIdx.x;
    const int64_t P = (int64_t)cands[c].nodes * cands[c].gpus;
    const unsigned long long* src = per_proc + proc_off[c] * 3;
    unsigned long long t[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
        for (int m = 0; m < 3; ++m) {
            const unsigned long long v = src[p * 3 + m];
            t[m] += v;
            mx[m] = v > mx[m] ? v : mx[m];
            if (out_per_proc) out_per_proc[(proc_off[c] + p) * 3 + m] = (int64_t)v;
        }
    }
    for (int m = 0; m < 3; ++m) {
        st[m][threadIdx.x] = t[m];
        sm[m][threadIdx.x] = mx[m];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int m = 0; m < 3; ++m) {
                st[m][threadIdx.x] += st[m][threadIdx.x + w];
                sm[m][threadIdx.x] = sm[m][threadIdx.x + w] > sm[m][threadIdx.x] ? sm[m][threadIdx.x + w]
                                                                                  : sm[m][threadIdx.x];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tm_matmul_cost r;
        for (int m = 0; m < 3; ++m) {
            r.tiles[m] = (int64_t)st[m][0];
            r.max_tiles[m] = (int64_t)sm[m][0];
        }
        r.bytes = (r.tiles[0] + r.tiles[1] + r.tiles[2]) * tile_bytes;
        out[c] = r;
    }
}

hipError_t launch_matmul_finalize(const DevCand* cands, int64_t n, const int64_t* proc_off,
                                  const unsigned long long* per_proc, int64_t tile_bytes, tm_matmul_cost* out,
                                  int64_t* out_per_proc, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_matmul_finalize, dim3((unsigned)n), dim3(256), 0, s, cands, proc_off, per_proc,
                       tile_bytes, out, out_per_proc);
    return hipGetLastError();
}

}  // namespace tmk
