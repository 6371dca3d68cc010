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

// Sum over the wave of non-negative per-lane counts, in 64 bits (a wave's counts for
// one work item can exceed 2^31 on very long rows).
__device__ __forceinline__ unsigned long long wave_sum64(int v) {
    unsigned long long s = (unsigned long long)(unsigned)v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// ------------------------------------------------------------------ table build

// One workgroup per candidate (grid-stride over candidates).  With halos (use_halo),
// each coordinate x of launch dim d gets the number of distinct non-zero offsets
// C_d[x +- s] - C_d[x] (1 <= s <= h_d, in-domain neighbours) in its entry, and for
// the last launch dim the list of those offsets.
__global__ __launch_bounds__(256) void k_build_tables(const DevHeader* __restrict__ hdr,
                                                      const DevCand* __restrict__ cands,
                                                      int32_t* __restrict__ arena, int use_halo) {
    __shared__ DevCand sc;
    const int64_t n = hdr->n;
    for (int64_t ci = blockIdx.x; ci < n; ci += gridDim.x) {
        __syncthreads();
        stage_cand(&sc, &cands[ci]);
        __syncthreads();
        int32_t* base = arena + sc.arena_off;
        // node-level tables keep the node of each owner (GPU bits cleared): the
        // counting kernel then counts distinct other nodes per cell
        const int32_t keep = hdr->node_level ? ~((1 << sc.gbits) - 1) : -1;
        for (int32_t v = threadIdx.x; v < sc.vol; v += blockDim.x) base[v] = owner_key(sc, v) & keep;
        const int hs = sc.hstride;
        for (int d = 0; d < sc.lrank; ++d) {
            const int64_t l = sc.extent[d];
            const int h = use_halo ? hdr->halo[d] : 0;
            int32_t* ct = base + sc.coord_off[d];
            const bool last = d == sc.lrank - 1;
            int32_t* dl = base + sc.dl_off[d];
            for (int64_t x = threadIdx.x; x < l; x += blockDim.x) {
                const int32_t val = coord_value(sc, d, x);
                int32_t found[2 * kMaxHalo];
                int cnt = 0;
                for (int s = 1; s <= h; ++s) {
                    for (int dir = 0; dir < 2; ++dir) {
                        const int64_t xx = dir ? x + s : x - s;
                        if (xx < 0 || xx >= l) continue;
                        const int32_t dv = coord_value(sc, d, xx) - val;
                        if (dv == 0) continue;
                        bool seen = false;
                        for (int i = 0; i < cnt; ++i) seen = seen || (found[i] == dv);
                        if (!seen) found[cnt++] = dv;
                    }
                }
                if (last)  // only the last dim's lists are stored (outer dims use the tables)
                    for (int i = 0; i < hs; ++i) dl[x * hs + i] = i < cnt ? found[i] : 0;
                ct[x] = val | (cnt << kCntShift);
            }
            if (d == sc.lrank - 1)  // zero entries up to a multiple of 512 (scanned eight per lane)
                for (int64_t x = l + threadIdx.x; x < ((l + 511) & ~int64_t(511)); x += blockDim.x) ct[x] = 0;
            if (last && hs > 0) {
                // mark cells whose counts equal their left neighbour's (bits 28..31 of
                // the entries are otherwise zero): same contribution and offset list
                // (bit 28, every row), or single offsets pointing at each other (bit
                // 29, rows without outer offsets)
                __syncthreads();
                for (int64_t x = 1 + threadIdx.x; x < l; x += blockDim.x) {
                    const int32_t e = ct[x] & 0x0fffffff, ep = ct[x - 1] & 0x0fffffff;
                    const int n = (e >> kCntShift) & 0xf, np = (ep >> kCntShift) & 0xf;
                    if (n == 0) continue;
                    bool same = e == ep;
                    for (int i = 0; i < hs && same; ++i) same = dl[x * hs + i] == dl[(x - 1) * hs + i];
                    bool mirror = false;
                    if (!same && n == 1 && np == 1) {
                        const int32_t dv = dl[(x - 1) * hs];
                        mirror = dv == (e & kValMask) - (ep & kValMask) && dl[x * hs] == -dv;
                    }
                    if (same || mirror) ct[x] = e | (1 << (same ? kSameShift : kMirrorShift));
                }
            }
        }
    }
}

hipError_t launch_build_tables(const DevHeader* hdr, const DevCand* cands, int64_t n, int32_t* arena,
                               int32_t use_halo, hipStream_t s) {
    const int64_t grid = n < 65536 ? (n > 0 ? n : 1) : 65536;
    hipLaunchKernelGGL(k_build_tables, dim3((unsigned)grid), dim3(256), 0, s, hdr, cands, arena, use_halo);
    return hipGetLastError();
}

// ------------------------------------------------------------------ reset

__global__ void k_reset(DevHeader* hdr, unsigned long long* counter, tm_stencil_cost* out, int64_t cap) {
    const int64_t n = hdr->n < cap ? hdr->n : cap;
    int64_t* o = reinterpret_cast<int64_t*>(out);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 4 * n;
         i += (int64_t)gridDim.x * blockDim.x)
        o[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0ull;
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
// A work item is a block of consecutive rows (all launch dims but the last fixed)
// of one candidate.  A workgroup takes items from a global atomic counter (the
// next one is requested while the current one runs), stages the candidate's owner
// table and, when they fit, the last dim's coordinate table and offset lists in LDS
// when the candidate changes (the outer dims' tables are read from global memory),
// and gives each wave every fourth row of the item, in batches of 64 rows whose
// fast outer entries and offsets one lane each works out at once, stepping the
// outer coordinates without divisions.  Every cell of every row is read and
// tested: a lane reads the coordinate entries of eight consecutive cells with two
// LDS loads, and the test (does the row hold cells with last-dim offsets) gates
// what follows.
//   - A row's outer coordinates fix its base index and the distinct non-zero
//     offsets to its outer neighbours, computed from the coordinate tables when
//     the row lies within a halo of a block boundary of an outer dim.
//   - Rows without outer offsets: a cell can have a foreign neighbour only along
//     the last dim, i.e. when its entry's offset count is non-zero.  In rows of
//     one chunk such cells form runs with equal results (listed once per row
//     range); consecutive such rows run in a tight loop.  With 8 or more runs a row
//     evaluates its runs at once, one per lane, and a row with the same base index
//     as the previous one reuses each lane's share; with fewer, rows queue their
//     base index and a drain evaluates the runs of several rows together.  Longer
//     rows compact their flagged cells into a per-wave LDS queue (prefix count from
//     ballots), evaluated 64 at a time; a chunk holding more than 64 of them is
//     evaluated in place.
//   - Rows with outer offsets: every cell counts.  Cells with equal results share
//     one evaluation: a stretch of equal entries without last-dim offsets (same
//     index, same neighbours), or of flagged cells marked equal to their left
//     neighbour.  For rows of one chunk these runs are listed once per row range,
//     and a row evaluates each run once, one per lane, times its length; a row whose
//     offsets come from the slower outer dims only reuses the previous such row's
//     shares while its fast outer entry and the slower outer coordinates repeat.
// Evaluating a cell: its owner o = T[v], then the owners T[v + delta] over the row
// offsets and the cell's last-dim offsets; the distinct ones other than o are
// counted (and those on another node).  Lanes count in registers, waves reduce,
// and one 64-bit atomic per wave and item adds to the candidate's totals.

// Per-wave LDS arrays of kQueueCap words, qv and qx: the queue of flagged cells of
// long rows (drained 128 at a time, two per lane; a push adds <= 64), or, for rows of
// one chunk, the run maps (qx[0..128): runs of rows without outer offsets, qx[128..):
// flagged runs and qv[128..): interior runs of rows with them).
constexpr int kQueueCap = 256;
constexpr int kCellsPerLane = 8;
constexpr int kChunk = 64 * kCellsPerLane;

__device__ __forceinline__ int32_t cval(int32_t e) { return e & kValMask; }
__device__ __forceinline__ int32_t ccnt(int32_t e) { return (e >> kCntShift) & 0xf; }

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Distinct owners, other than o, among T[v + delta] for delta in rl[0..nr) then
// xl[0..nx).  Offsets are distinct within each list; equal owners are merged.
// The first two owners are handled in straight-line code (the usual case).
template <typename XP>
__device__ __forceinline__ void eval_cell(const int32_t* __restrict__ T, int32_t v, const int32_t* rl, int nr,
                                          XP xl, int nx, int gbits, int& cnt, int& icnt) {
    const int n = nr + nx;
    if (n == 0) return;
    const int32_t o = T[v];
    const int32_t onode = o >> gbits;
    const int32_t d0 = nr > 0 ? rl[0] : xl[0];
    const int32_t o0 = T[v + d0];
    const bool f0 = o0 != o;
    cnt += f0;
    icnt += (f0 && (o0 >> gbits) != onode) ? 1 : 0;
    if (n == 1) return;
    const int32_t d1 = nr > 1 ? rl[1] : xl[1 - nr];
    const int32_t o1 = T[v + d1];
    const bool f1 = o1 != o && o1 != o0;
    cnt += f1;
    icnt += (f1 && (o1 >> gbits) != onode) ? 1 : 0;
    for (int t = 2; t < n; ++t) {
        const int32_t dt = t < nr ? rl[t] : xl[t - nr];
        const int32_t ot = T[v + dt];
        bool fresh = ot != o && ot != o0 && ot != o1;
        for (int s = 2; s < t && fresh; ++s) {
            const int32_t ds = s < nr ? rl[s] : xl[s - nr];
            fresh = T[v + ds] != ot;
        }
        if (fresh) {
            ++cnt;
            icnt += ((ot >> gbits) != onode) ? 1 : 0;
        }
    }
}

// Evaluates the cells x0 .. x0+7 of a row (see above).  only_flagged: skip cells
// without last-dim offsets (rows without outer offsets).
template <int32_t SAME, typename XP>
__device__ __forceinline__ void eval_group(const int32_t* __restrict__ T, XP DL, int HS,
                                           const int32_t (&e8)[kCellsPerLane], int x0, int L, int32_t base,
                                           const int32_t* rl, int nr, int gbits, bool only_flagged, int& cnt,
                                           int& icnt) {
    int32_t ep = -1;  // never a valid entry (bits 29..31 are zero)
    int cp = 0, ip = 0;
#pragma unroll
    for (int j = 0; j < kCellsPerLane; ++j) {
        const int x = x0 + j;
        const int32_t e = e8[j];
        const int nx = ccnt(e);
        if (x >= L || (only_flagged && nx == 0)) continue;
        // a flagged cell whose entry carries one of the SAME bits has the result of
        // its left neighbour (evaluated just before, in this lane)
        const bool same = SAME != 0 && j > 0 && (e & SAME) != 0;
        if (!same && (e != ep || nx != 0)) {
            cp = 0;
            ip = 0;
            eval_cell(T, base + cval(e), rl, nr, DL + x * HS, nx, gbits, cp, ip);
            ep = nx == 0 ? e : -1;
        }
        cnt += cp;
        icnt += ip;
    }
}

// Distinct owners, other than T[v], among T[v + rl[t]] for t < nr (nr >= 1).
__device__ __forceinline__ void eval_row_offsets(const int32_t* __restrict__ T, int32_t v, const int32_t* rl, int nr,
                                                 int gbits, int& cnt, int& icnt) {
    const int32_t o = T[v];
    const int32_t onode = o >> gbits;
    const int32_t o0 = T[v + rl[0]];
    const int32_t o1 = T[v + (nr > 1 ? rl[1] : 0)];
    const bool f0 = o0 != o;
    const bool f1 = o1 != o && o1 != o0;
    cnt += (int)f0 + (int)f1;
    icnt += (f0 && (o0 >> gbits) != onode ? 1 : 0) + (f1 && (o1 >> gbits) != onode ? 1 : 0);
    for (int t = 2; t < nr; ++t) {
        const int32_t ot = T[v + rl[t]];
        bool fresh = ot != o && ot != o0 && ot != o1;
        for (int s2 = 2; s2 < t && fresh; ++s2) fresh = T[v + rl[s2]] != ot;
        if (fresh) {
            ++cnt;
            icnt += ((ot >> gbits) != onode) ? 1 : 0;
        }
    }
}

// One queued cell (row base index bq, last-dim coordinate xq) of a row without
// outer offsets: only its last-dim neighbours can be foreign.  The first two
// offsets are loaded without branches (a cell's list always has HS >= 2 slots;
// unused offsets are replaced by 0, which reads the cell's own owner), so the
// owner lookups of the usual one- and two-offset cells issue together.
template <typename XP>
__device__ __forceinline__ void eval_queued(const int32_t* __restrict__ T, const int32_t* __restrict__ CL, XP DL,
                                            int HS, int32_t bq, int32_t xq, int gbits, int& cnt, int& icnt) {
    const int32_t e = CL[xq];
    const int32_t d0 = DL[xq * HS], d1 = DL[xq * HS + 1];
    const int32_t v = bq + cval(e);
    const int nx = ccnt(e);
    const int32_t o = T[v];
    const int32_t o0 = T[v + (nx > 0 ? d0 : 0)];
    const int32_t o1 = T[v + (nx > 1 ? d1 : 0)];
    const int32_t onode = o >> gbits;
    const bool f0 = o0 != o;
    const bool f1 = o1 != o && o1 != o0;
    cnt += (int)f0 + (int)f1;
    icnt += (f0 && (o0 >> gbits) != onode ? 1 : 0) + (f1 && (o1 >> gbits) != onode ? 1 : 0);
    for (int t = 2; t < nx; ++t) {
        const int32_t ot = T[v + DL[xq * HS + t]];
        bool fresh = ot != o && ot != o0 && ot != o1;
        for (int s2 = 2; s2 < t && fresh; ++s2) fresh = T[v + DL[xq * HS + s2]] != ot;
        if (fresh) {
            ++cnt;
            icnt += ((ot >> gbits) != onode) ? 1 : 0;
        }
    }
}

// Number of set bits of m in the lanes below this one.
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Flags of a lane's eight cells (bit j: cell j has last-dim offsets), the number of
// flagged cells in the lanes below (prefix over the wave, from the ballots of the
// four bit planes of the per-lane counts 0..8) and the wave's total.
__device__ __forceinline__ void chunk_flags(const int32_t (&e8)[kCellsPerLane], uint32_t& fl, int& pre, int& tot) {
    fl = 0;
#pragma unroll
    for (int j = 0; j < kCellsPerLane; ++j) fl |= ((uint32_t)e8[j] > (uint32_t)kValMask ? 1u : 0u) << j;
    const int c = __popc(fl);
    pre = 0;
    tot = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint64_t m = __ballot((c >> b) & 1);
        pre += lanes_below(m) << b;
        tot += __popcll(m) << b;
    }
}

__device__ __forceinline__ void load8(const int32_t* p, int32_t (&e8)[kCellsPerLane]) {
    const i32x4 a = *reinterpret_cast<const i32x4*>(p);
    const i32x4 b = *reinterpret_cast<const i32x4*>(p + 4);
    e8[0] = a.x;
    e8[1] = a.y;
    e8[2] = a.z;
    e8[3] = a.w;
    e8[4] = b.x;
    e8[5] = b.y;
    e8[6] = b.z;
    e8[7] = b.w;
}

// Distinct non-zero offsets from coordinate q of outer dim d to its in-domain
// neighbours within the halo, appended to rl[nr..) (uniform: every lane writes the
// same values).  Offsets equal to the previous one in the same direction are
// dropped (a block holds consecutive coordinates).
template <int H>
__device__ __forceinline__ int outer_offsets(const int32_t* __restrict__ C, int32_t q, int32_t ext, int h,
                                             int32_t* rl, int nr) {
    const int32_t ev = cval(C[q]);
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        int32_t prev = 0;
#pragma unroll
        for (int s = 1; s <= H; ++s) {
            const int32_t xx = dir ? q + s : q - s;
            if (s <= h && xx >= 0 && xx < ext) {
                const int32_t dv = cval(C[xx]) - ev;
                if (dv != 0 && dv != prev) rl[nr++] = dv;
                prev = dv;
            }
        }
    }
    return nr;
}

// The rows [ra, rb) of the staged candidate, for one wave.
template <int K, int H, typename XP>
__device__ __forceinline__ void count_rows(const int32_t* __restrict__ T, const int32_t* __restrict__ G,
                                           const int32_t* __restrict__ CL, XP DL,
                                           const int32_t (&off)[K], const int32_t (&ext)[K], const int (&hal)[K],
                                           int32_t ra, int32_t rb, int rs, int L, int gbits, int lane, int32_t* rl,
                                           int32_t* qv, int32_t* qx, int32_t* ob, int& cnt, int& icnt) {
    constexpr int HS = 2 * H;
    constexpr int KO = K > 1 ? K - 1 : 1;
    int qn = 0;  // wave-uniform queue length
    // Rows that fit one chunk: in rows without outer offsets the flags of a lane's
    // cells depend on the last coordinate only, so their compaction (per-lane
    // flags, prefix over the wave, total) is computed once here.
    const bool one_chunk = L <= kChunk;
    uint32_t hfl = 0, rfl = 0, dfl = 0, ifl = 0;
    int hpre = 0, htot = 0, rpre = 0, rtot = 0, dpre = 0, dtot = 0, ipre = 0, itot = 0;
    if (one_chunk) {
        int32_t e8[kCellsPerLane];
        load8(CL + kCellsPerLane * lane, e8);
        chunk_flags(e8, hfl, hpre, htot);
        // runs: a flagged cell whose counts equal its left neighbour's has that
        // neighbour's result; only run starts are kept -- rfl for rows without outer
        // offsets (either bit), dfl for rows with them (equal entries only)
#pragma unroll
        for (int j = 0; j < kCellsPerLane; ++j) {
            const bool f = (hfl >> j) & 1u;
            rfl |= (f && !((e8[j] >> kSameShift) & 3) ? 1u : 0u) << j;
            dfl |= (f && !((e8[j] >> kSameShift) & 1) ? 1u : 0u) << j;
            // interior runs: cells without last-dim offsets, a run per maximal stretch
            // of equal entries (same index, same neighbours in every row)
            const int32_t x = kCellsPerLane * lane + j;
            const int32_t el = j > 0 ? e8[j - 1] : (lane > 0 ? CL[x - 1] : -1);
            ifl |= (x < L && !f && e8[j] != el ? 1u : 0u) << j;
        }
        const int ci = __popc(ifl);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint64_t mi = __ballot((ci >> b) & 1);
            ipre += lanes_below(mi) << b;
            itot += __popcll(mi) << b;
        }
        const int c = __popc(rfl), cd = __popc(dfl);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint64_t m = __ballot((c >> b) & 1), md = __ballot((cd >> b) & 1);
            rpre += lanes_below(m) << b;
            rtot += __popcll(m) << b;
            dpre += lanes_below(md) << b;
            dtot += __popcll(md) << b;
        }
    }
    // Row queue (single-chunk rows with 1..128 runs of flagged cells): a row without
    // outer offsets queues only its base index (lane i of qrow holds that of queued
    // row i, fetched in the drain with a lane permute); a drain of rq_rows rows evaluates
    // rq_rows * rtot <= 128 run starts, entry idx being run idx % rtot of queued row
    // idx / rtot, each counted times its run length.  qx[0..128) holds that map as
    // (run length << 18) | (x << 8) | row, built once here (staged in qx[128..256));
    // qx[128..128 + dtot) then holds the flagged runs of rows with outer offsets and
    // qv[128..128 + itot) their interior runs (rowd: when there are at most 128 of
    // each; else such rows take the general dense path).
    const bool rowq = one_chunk && rtot > 0 && rtot <= 128;
    const bool fastq = one_chunk && rtot <= 128;  // rows without outer offsets in the tight loop (rowq, or no runs)
    const bool rowd = one_chunk && dtot <= 128 && itot <= 128;
    const int rq_rows = rowq ? (rtot == 1 ? 64 : 128 / rtot) : 0;  // at most 64: one row base per lane
    const int rq_cells = rq_rows * rtot;
    int nrow = 0;
    if (rowq || rowd) {
        auto stage_runs = [&](uint32_t f, int pos, int32_t bits) {
            while (f) {
                const int j = __builtin_ctz(f);
                f &= f - 1;
                const int32_t x = kCellsPerLane * lane + j;
                int32_t run = 1;
                while (x + run < L && (CL[x + run] & bits) != 0) ++run;
                qx[pos++] = x | (run << 10);
            }
        };
        if (rowd) {  // interior runs to qv[128..128 + itot): (len << 18) | (x << 8)
            uint32_t f = ifl;
            int pos = 128 + ipre;
            while (f) {
                const int j = __builtin_ctz(f);
                f &= f - 1;
                const int32_t x = kCellsPerLane * lane + j;
                const int32_t e = CL[x];
                int32_t run = 1;
                while (x + run < L && CL[x + run] == e) ++run;
                qv[pos++] = (x << 8) | (run << 18);
            }
        }
        if (rowq) {
            stage_runs(rfl, 128 + rpre, 3 << kSameShift);
            wave_sync_lds();
            int32_t m0 = 0, m1 = 0;
            if (lane < rq_cells) {
                const int r = lane / rtot;
                m0 = (qx[128 + lane - r * rtot] << 8) | r;
            }
            if (lane + 64 < rq_cells) {
                const int r = (lane + 64) / rtot;
                m1 = (qx[128 + lane + 64 - r * rtot] << 8) | r;
            }
            wave_sync_lds();
            if (lane < rq_cells) qx[lane] = m0;
            if (lane + 64 < rq_cells) qx[lane + 64] = m1;
        }
        if (rowd) {
            stage_runs(dfl, 128 + dpre, 1 << kSameShift);
            wave_sync_lds();
            if (lane < dtot) qx[128 + lane] <<= 8;
            if (lane + 64 < dtot) qx[192 + lane] <<= 8;
        }
        wave_sync_lds();
    }
    auto run_x = [](int32_t m) { return (m >> 8) & 0x3ff; };
    auto run_len = [](int32_t m) { return (m >> 18) & 0x3ff; };
    // queued row bases: lane i holds that of queued row i
    int32_t qrow = 0;
    auto drain_rows = [&](int ncell) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int idx = lane + 64 * half;
            const int32_t m = qx[idx];
            // every lane takes part in the permute (entries past ncell are not used)
            const int32_t bq = __builtin_amdgcn_ds_bpermute((m & 63) << 2, qrow);
            if (idx < ncell) {
                int c = 0, ic = 0;
                eval_queued(T, CL, DL, HS, bq, run_x(m), gbits, c, ic);
                cnt += run_len(m) * c;
                icnt += run_len(m) * ic;
            }
        }
    };
    int32_t q[KO];
    {
        uint32_t rr = (uint32_t)ra;
#pragma unroll
        for (int d = K - 2; d >= 0; --d) {
            q[d] = (int32_t)(rr % (uint32_t)ext[d]);
            rr /= (uint32_t)ext[d];
        }
    }
    // prefix over dims 0..K-3: base index and offsets, refreshed on carries
    int32_t base_o = 0;
    int no = 0;
    // the last row with outer offsets from dims 0..K-3 only: its dim K-2 entry, and
    // each lane's share of its counts (rows with the same entry under the same
    // prefix have the same index and neighbours)
    int32_t dkey = -1;
    bool dflag = false;
    int dmc = 0, dmic = 0;
    auto load_prefix = [&]() {
        base_o = 0;
        no = 0;
        dkey = -1;
#pragma unroll
        for (int d = 0; d < K - 2; ++d) {
            const int32_t e = uniform32(G[off[d] + q[d]]);
            base_o += cval(e);
            if (ccnt(e)) no = outer_offsets<H>(G + off[d], q[d], ext[d], hal[d], rl, no);
        }
    };
    load_prefix();
    // entries of dim K-2 for this wave's next 64 rows, one per lane (lane i: the row
    // i steps of rs ahead), so a row takes its entry with a lane read instead of a
    // memory round trip.  A lane also works out its row's offsets along dim K-2 (the
    // rule of outer_offsets, neighbour entries loaded together): the first two go to
    // ob[2i], ob[2i+1], their number to bits 28..31 of the entry (15: more than two,
    // left to outer_offsets).
    int32_t eb = 0;
    auto load_batch = [&]() {
        if constexpr (K > 1) {
            const int32_t* C = G + off[K - 2];
            const int32_t qi = (int32_t)((uint32_t)(q[K - 2] + lane * rs) % (uint32_t)ext[K - 2]);
            eb = C[qi];
            if (ccnt(eb)) {
                const int32_t ev = cval(eb);
                int c = 0;
                int32_t o0 = 0, o1 = 0;
#pragma unroll
                for (int dir = 0; dir < 2; ++dir) {
                    int32_t prev = 0;
#pragma unroll
                    for (int s = 1; s <= H; ++s) {
                        const int32_t xx = dir ? qi + s : qi - s;
                        if (s <= hal[K - 2] && xx >= 0 && xx < ext[K - 2]) {
                            const int32_t dv = cval(C[xx]) - ev;
                            if (dv != 0 && dv != prev) {
                                if (c == 0) o0 = dv;
                                if (c == 1) o1 = dv;
                                ++c;
                            }
                            prev = dv;
                        }
                    }
                }
                ob[2 * lane] = o0;
                ob[2 * lane + 1] = o1;
                eb |= (c > 2 ? 15 : c) << 28;
            }
            wave_sync_lds();
        }
    };
    // the wave's rows ra, ra + rs, ... below rb, in batches of up to 64
    const int nrows = (rb - ra + rs - 1) / rs;
    // sparse single-chunk row: every cell is read and tested; the row's flagged cells
    // are the precomputed ones, so only its base is queued
    // Rows with several runs (crowd: 8 or more) are evaluated at once, one run per
    // lane, and a row with the same base index as the previous one of this wave (the
    // same outer blocks) has the same result: each lane adds its share again.  Rows
    // with fewer runs go to the row queue, which fills the lanes from several rows.
    const bool crowd = rtot >= 8;
    int32_t mbase = -1, mc = 0, mic = 0;
    auto sparse_row = [&](int32_t base) {
        int32_t e8[kCellsPerLane];
        load8(CL + kCellsPerLane * lane, e8);
        int32_t any = 0;
#pragma unroll
        for (int j = 0; j < kCellsPerLane; ++j) any |= e8[j];
        if (__ballot((uint32_t)any > (uint32_t)kValMask) == 0ull) return;
        if (crowd) {
            if (base != mbase) {
                mc = 0;
                mic = 0;
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int k = lane + 64 * half;
                    if (k < rtot) {
                        const int32_t m = qx[k];  // run k of map row 0
                        int c = 0, ic = 0;
                        eval_queued(T, CL, DL, HS, base, run_x(m), gbits, c, ic);
                        mc += run_len(m) * c;
                        mic += run_len(m) * ic;
                    }
                }
                mbase = base;
            }
            cnt += mc;
            icnt += mic;
        } else {
            qrow = lane == nrow ? base : qrow;
            ++nrow;
            if (nrow == rq_rows) {
                wave_sync_lds();
                drain_rows(rq_cells);
                wave_sync_lds();
                nrow = 0;
            }
        }
    };
    // next row of this wave (row index i of nrows): step the outer coordinates by rs,
    // carried into the outer dims only while rows remain, so they never leave the domain
    auto step_row = [&](int i) {
        if constexpr (K > 1) {
            q[K - 2] += rs;
            if (__builtin_expect(q[K - 2] >= ext[K - 2], 0) && i + 1 < nrows) {
                int32_t c = 0;
                while (q[K - 2] >= ext[K - 2]) {
                    q[K - 2] -= ext[K - 2];
                    ++c;
                }
#pragma unroll
                for (int d = K - 3; d >= 0; --d) {
                    q[d] += c;
                    c = 0;
                    while (q[d] >= ext[d]) {
                        q[d] -= ext[d];
                        ++c;
                    }
                }
                load_prefix();
                wave_sync_lds();
            }
        }
    };
    for (int done = 0; done < nrows; done += 64) {
      load_batch();
      const int nb = nrows - done < 64 ? nrows - done : 64;
      for (int tb = 0; tb < nb; ++tb) {
        if constexpr (K > 1) {
            // consecutive rows without outer offsets (the common case) in a tight loop
            // (with no runs, a row only has its cells read and tested); the first row
            // with offsets falls through to the general code below
            if (fastq && no == 0) {
                while (tb < nb) {
                    const int32_t e = __builtin_amdgcn_readlane(eb, tb);
                    if (ccnt(e)) break;
                    sparse_row(base_o + cval(e));
                    ++tb;
                    q[K - 2] += rs;
                    if (q[K - 2] >= ext[K - 2]) {  // a carry: the general code takes the next row
                        q[K - 2] -= rs;
                        step_row(done + tb - 1);
                        break;
                    }
                }
                if (tb == nb) break;
            }
        }
        int32_t base = base_o;
        int nr = no;
        int32_t erow = -1;  // dim K-2 entry of a row whose offsets come from the prefix only
        if constexpr (K > 1) {
            const int32_t e = __builtin_amdgcn_readlane(eb, tb);
            if (ccnt(e) == 0) erow = e;
            base += cval(e);
            if (ccnt(e)) {
                const int c = (int)((uint32_t)e >> 28);
                if (c <= 2) {
                    rl[no] = ob[2 * tb];
                    rl[no + 1] = ob[2 * tb + 1];
                    nr = no + c;
                } else {
                    nr = outer_offsets<H>(G + off[K - 2], q[K - 2], ext[K - 2], hal[K - 2], rl, no);
                }
            }
        }
        if (nr == 0) {
          if (rowq) {
            sparse_row(base);
          } else {
            // ---- sparse row: cells with last-dim offsets go to the queue one by one
            for (int xb = 0; xb < L; xb += kChunk) {
                const int x0 = xb + kCellsPerLane * lane;
                int32_t e8[kCellsPerLane];
                load8(CL + x0, e8);  // zero-padded past L
                int32_t any = 0;
#pragma unroll
                for (int j = 0; j < kCellsPerLane; ++j) any |= e8[j];
                const bool hit = (uint32_t)any > (uint32_t)kValMask;
                if (__ballot(hit) == 0ull) continue;
                uint32_t fl = hfl;
                int pre = hpre, tot = htot;
                if (!one_chunk) chunk_flags(e8, fl, pre, tot);
                if (tot > 64) {  // a crowded chunk: evaluate it in place
                    eval_group<(H > 1 ? 3 << kSameShift : 0)>(T, DL, HS, e8, x0, L, base, rl, 0, gbits, true,
                                                               cnt, icnt);
                    continue;
                }
                int pos = qn + pre;
                while (fl) {
                    const int j = __builtin_ctz(fl);
                    fl &= fl - 1;
                    qv[pos] = base;
                    qx[pos] = x0 + j;
                    ++pos;
                }
                qn += tot;
                wave_sync_lds();
                if (qn >= 128) {
                    eval_queued(T, CL, DL, HS, qv[lane], qx[lane], gbits, cnt, icnt);
                    eval_queued(T, CL, DL, HS, qv[lane + 64], qx[lane + 64], gbits, cnt, icnt);
                    wave_sync_lds();
                    if (lane < qn - 128) {
                        qv[lane] = qv[lane + 128];
                        qx[lane] = qx[lane + 128];
                    }
                    qn -= 128;
                    wave_sync_lds();
                }
            }
          }
        } else {
            // ---- rows with outer offsets: every cell counts.  Every cell is read and
            // tested (whether the row holds flagged cells, which gates their runs and is
            // part of the memo's check); a row repeating the remembered entry under the
            // same prefix adds the remembered shares.
            int32_t e8[kCellsPerLane];
            load8(CL + kCellsPerLane * lane, e8);
            int32_t any = 0;
#pragma unroll
            for (int j = 0; j < kCellsPerLane; ++j) any |= e8[j];
            const bool has_flagged = __ballot((uint32_t)any > (uint32_t)kValMask) != 0ull;
            if (erow >= 0 && erow == dkey && has_flagged == dflag) {
                cnt += dmc;
                icnt += dmic;
            } else {
                int rc = 0, ric = 0;
                if (rowd) {
                    // single chunk: interior runs, then flagged runs, one per lane from the maps
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const int k = lane + 64 * half;
                        if (k < itot) {
                            const int32_t m = qv[128 + k];
                            int c = 0, ic = 0;
                            eval_row_offsets(T, base + cval(CL[run_x(m)]), rl, nr, gbits, c, ic);
                            rc += run_len(m) * c;
                            ric += run_len(m) * ic;
                        }
                    }
                    if (has_flagged) {
#pragma unroll
                        for (int half = 0; half < 2; ++half) {
                            const int k = lane + 64 * half;
                            if (k < dtot) {
                                const int32_t m = qx[128 + k];
                                const int32_t x = run_x(m);
                                const int32_t e = CL[x];
                                int c = 0, ic = 0;
                                eval_cell(T, base + cval(e), rl, nr, DL + x * HS, ccnt(e), gbits, c, ic);
                                rc += run_len(m) * c;
                                ric += run_len(m) * ic;
                            }
                        }
                    }
                } else {
                    // every chunk, eight cells per lane (memoised on equal entries)
                    for (int xb = 0; xb < L; xb += kChunk) {
                        const int x0 = xb + kCellsPerLane * lane;
                        if (x0 >= L) continue;
                        int32_t f8[kCellsPerLane];
                        load8(CL + x0, f8);
                        eval_group<(H > 1 ? 1 << kSameShift : 0)>(T, DL, HS, f8, x0, L, base, rl, nr, gbits, false,
                                                                   rc, ric);
                    }
                }
                cnt += rc;
                icnt += ric;
                if (erow >= 0) {
                    dkey = erow;
                    dflag = has_flagged;
                    dmc = rc;
                    dmic = ric;
                }
            }
            wave_sync_lds();
        }
        step_row(done + tb);
      }
    }
    // drain the queues
    if (nrow > 0) {
        wave_sync_lds();
        drain_rows(nrow * rtot);
        wave_sync_lds();
    }
    if (qn > 0) {
        if (lane < qn) eval_queued(T, CL, DL, HS, qv[lane], qx[lane], gbits, cnt, icnt);
        if (lane + 64 < qn) eval_queued(T, CL, DL, HS, qv[lane + 64], qx[lane + 64], gbits, cnt, icnt);
        wave_sync_lds();
    }
}

// Waves per SIMD: seven for H >= 2 and six for H = 1 (measured on the 512^3 halo-2
// workload and the random halo-1 batch: 5 / 6 / 7 / 8 waves 4.47 / 4.02 / 3.89 /
// 3.94 ms at H = 2; 4 / 5 / 6 / 7 waves 19.4 / 16.5 / 15.1 / 15.4 ms at H = 1); the
// compiler then spills a few registers to scratch, which these times include.
template <int K, int H>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(H == 1 ? 6 : 7))) void k_count(const DevHeader* __restrict__ hdr,
                                               const DevCand* __restrict__ cands,
                                               const int32_t* __restrict__ arena,
                                               unsigned long long* __restrict__ counter,
                                               tm_stencil_cost* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // 16-byte aligned: ds_read_b128 of staged tables
    __shared__ long long s_item;
    __shared__ int32_t s_qv[4][kQueueCap], s_qx[4][kQueueCap];
    __shared__ int32_t s_rl[4][32];
    __shared__ int32_t s_ob[4][128];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps the row loops scalar
    const int64_t total = uniform64(hdr->total_items);
    const int64_t n = uniform64(hdr->n);
    int hal[K];
#pragma unroll
    for (int d = 0; d < K; ++d) hal[d] = uniform32(hdr->halo[d]);

    int64_t cur = -1;
    int32_t L = 0, gbits = 0, rpi = 1, dl_lds = 0;
    int64_t rows = 0, ifirst = 0;
    int32_t off[K], ext[K];
    int32_t dlo = 0;
    const int32_t* garena = arena;
#pragma unroll
    for (int d = 0; d < K; ++d) off[d] = ext[d] = 0;

    unsigned long long next = 0;
    if (tid == 0) next = atomicAdd(counter, 1ull);
    for (;;) {
        if (tid == 0) s_item = (long long)next;
        __syncthreads();
        const int64_t item = uniform64(s_item);
        __syncthreads();
        if (item >= total) break;
        if (tid == 0) next = atomicAdd(counter, 1ull);

        // candidate owning this item (binary search over item_first)
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (cands[mid].item_first <= item) lo = mid;
            else hi = mid - 1;
        }
        lo = uniform64(lo);
        if (lo != cur) {
            const DevCand* c = &cands[lo];
            const int32_t words = uniform32(c->lds_words);
            const int32_t* src = arena + c->arena_off;
            for (int i = tid; i < words; i += 256) lds[i] = src[i];
            garena = src;
            L = uniform32(c->L);
            gbits = uniform32(c->gbits);
            rpi = uniform32(c->rows_per_item);
            rows = uniform64(c->rows);
            ifirst = uniform64(c->item_first);
#pragma unroll
            for (int d = 0; d < K; ++d) {
                off[d] = uniform32(c->coord_off[d]);
                ext[d] = uniform32((int32_t)c->extent[d]);
            }
            dlo = uniform32(c->dl_off[K - 1]);
            dl_lds = uniform32(c->dl_lds);
            cur = lo;
            __syncthreads();
        }
        // this wave's rows of the item: every fourth, so rows near block boundaries
        // (dense ones cluster there) spread evenly over the waves
        // rows of a candidate fit 31 bits (checked on the host)
        const int32_t r0 = (int32_t)(item - ifirst) * rpi;
        const int32_t rb = (int64_t)r0 + rpi < rows ? r0 + rpi : (int32_t)rows;
        const int32_t ra = r0 + wid;
        int cnt = 0, icnt = 0;
        if (ra < rb) {
            if (dl_lds)  // last dim's table and offset lists in LDS
                count_rows<K, H>(lds, garena, lds + off[K - 1], lds + dlo, off, ext, hal, ra, rb, 4, L, gbits, lane,
                                 s_rl[wid], s_qv[wid], s_qx[wid], s_ob[wid], cnt, icnt);
            else  // long rows: both read from global memory (one code path keeps the kernel small)
                count_rows<K, H>(lds, garena, garena + off[K - 1], garena + dlo, off, ext, hal, ra, rb, 4, L, gbits,
                                 lane, s_rl[wid], s_qv[wid], s_qx[wid], s_ob[wid], cnt, icnt);
        }
        const unsigned long long c64 = wave_sum64(cnt), i64 = wave_sum64(icnt);
        if (lane == 0 && (c64 | i64)) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].ghost_cells), c64);
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].inter_cells), i64);
        }
    }
}

template <int K, int H>
static void* count_fn() {
    return reinterpret_cast<void*>(&k_count<K, H>);
}

static void* pick_count(int K, int H) {
#define TM_PICK(k)                              \
    if (K == k) {                               \
        if (H == 1) return count_fn<k, 1>();    \
        if (H == 2) return count_fn<k, 2>();    \
        if (H == 3) return count_fn<k, 3>();    \
        if (H == 4) return count_fn<k, 4>();    \
    }
    TM_PICK(1) TM_PICK(2) TM_PICK(3) TM_PICK(4)
#undef TM_PICK
    return nullptr;
}

int count_kernel_occupancy(int K, int H, int lds_words, int* blocks_per_cu) {
    void* fn = pick_count(K, H);
    if (!fn) return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, (size_t)lds_words * 4) != hipSuccess)
        return -1;
    *blocks_per_cu = nb;
    return 0;
}

hipError_t launch_count(int K, int H, const DevHeader* hdr, const DevCand* cands, const int32_t* arena,
                        unsigned long long* counter, tm_stencil_cost* out, int grid, int lds_words,
                        hipStream_t s) {
    void* fn = pick_count(K, H);
    if (!fn) return hipErrorInvalidValue;
    void* args[] = {(void*)&hdr, (void*)&cands, (void*)&arena, (void*)&counter, (void*)&out};
    return hipLaunchKernel(fn, dim3(grid), dim3(256), args, (size_t)lds_words * 4, s);
}

// ------------------------------------------------------------------ bytes + selection

// One workgroup: bytes from cell counts, then the minimum of (bytes, inter_bytes, index).
__global__ __launch_bounds__(1024) void k_finalize_select(const DevHeader* __restrict__ hdr,
                                                          tm_stencil_cost* __restrict__ out,
                                                          int64_t* __restrict__ best) {
    __shared__ int64_t sb[1024], si[1024], sx[1024];
    const int64_t n = hdr->n;
    const int64_t eb = hdr->elem_bytes;
    int64_t kb = INT64_MAX, ki = INT64_MAX, kx = INT64_MAX;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        tm_stencil_cost c = out[i];
        c.bytes = c.ghost_cells * eb;
        c.inter_bytes = c.inter_cells * eb;
        out[i] = c;
        if (c.bytes < kb || (c.bytes == kb && (c.inter_bytes < ki || (c.inter_bytes == ki && i < kx)))) {
            kb = c.bytes;
            ki = c.inter_bytes;
            kx = i;
        }
    }
    sb[threadIdx.x] = kb;
    si[threadIdx.x] = ki;
    sx[threadIdx.x] = kx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const int o = threadIdx.x + w;
            if (sb[o] < sb[threadIdx.x] ||
                (sb[o] == sb[threadIdx.x] &&
                 (si[o] < si[threadIdx.x] || (si[o] == si[threadIdx.x] && sx[o] < sx[threadIdx.x])))) {
                sb[threadIdx.x] = sb[o];
                si[threadIdx.x] = si[o];
                sx[threadIdx.x] = sx[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && best) *best = n > 0 ? sx[0] : -1;
}

hipError_t launch_finalize_select(const DevHeader* hdr, tm_stencil_cost* out, int64_t* best, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_select, dim3(1), dim3(1024), 0, s, hdr, out, best);
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
// Rows of the launch domain are spread over the workgroups; each wave writes whole
// rows.  A lane produces four consecutive points (one 16-byte non-temporal store)
// when the row start is 16-byte aligned, else single points.  The owner table and
// (when it fits) the last dim's coordinate table sit in LDS; the outer dims'
// tables are read once per row from global memory.

__global__ __launch_bounds__(256) void k_map(const DevCand* __restrict__ cands, int64_t n,
                                             const int32_t* __restrict__ arena,
                                             const int64_t* __restrict__ d_index, int64_t index,
                                             int32_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // 16-byte aligned: ds_read_b128 of staged tables
    __shared__ DevCand sc;
    const int64_t ci = d_index ? uniform64(*d_index) : index;
    if (ci < 0 || ci >= n) return;  // no candidate selected (empty batch)
    stage_cand(&sc, &cands[ci]);
    __syncthreads();
    const int32_t words = sc.lds_words;
    const int32_t* src = arena + sc.arena_off;
    for (int i = threadIdx.x; i < words; i += blockDim.x) lds[i] = src[i];
    __syncthreads();

    const int K = sc.lrank;
    const int32_t L = sc.L;
    const int64_t rows = sc.rows;
    const int32_t gb = sc.gbits, g = sc.gpus, gmask = (1 << sc.gbits) - 1;
    const int32_t* T = lds;
    const int32_t* G = arena + sc.arena_off;  // outer tables (and a last-dim table that did not fit)
    const int32_t* CL = sc.cl_lds ? lds + sc.coord_off[K - 1] : G + sc.coord_off[K - 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const bool vec = (L & 3) == 0 && ((reinterpret_cast<uintptr_t>(out) & 15) == 0);
    // a wave's rows are r0 + t * nw; lane i works out the base index of row
    // r0 + i * nw for 64 rows at a time, and row t takes it with a lane read
    const int64_t r0 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(wid);
    int32_t bl = 0;
    for (int64_t t = 0, r = r0; r < rows; ++t, r += nw) {
        if ((t & 63) == 0) {
            const int64_t ri = r + (int64_t)lane * nw;
            bl = 0;
            if (ri < rows) {
                uint32_t rr = (uint32_t)ri;
                for (int d = K - 2; d >= 0; --d) {
                    const uint32_t e = (uint32_t)sc.extent[d];
                    bl += G[sc.coord_off[d] + (int32_t)(rr % e)] & kValMask;
                    rr /= e;
                }
            }
        }
        const int32_t base = __builtin_amdgcn_readlane(bl, (int)(t & 63));
        int32_t* row = out + r * (int64_t)L;
        if (vec) {
            for (int x = lane * 4; x < L; x += 256) {
                i32x4 key;
                key.x = T[base + (CL[x] & kValMask)];
                key.y = T[base + (CL[x + 1] & kValMask)];
                key.z = T[base + (CL[x + 2] & kValMask)];
                key.w = T[base + (CL[x + 3] & kValMask)];
                const i32x4 p = (key >> gb) * g + (key & gmask);
                __builtin_nontemporal_store(p, reinterpret_cast<i32x4*>(row + x));
            }
        } else {
            for (int x = lane; x < L; x += 64) {
                const int32_t key = T[base + (CL[x] & kValMask)];
                __builtin_nontemporal_store((key >> gb) * g + (key & gmask), row + x);
            }
        }
    }
}

hipError_t launch_map(const DevCand* cands, int64_t n, const int32_t* arena, const int64_t* d_index,
                      int64_t index, int32_t* out, int grid, int lds_words, hipStream_t s) {
    hipLaunchKernelGGL(k_map, dim3(grid), dim3(256), (size_t)lds_words * 4, s, cands, n, arena, d_index, index,
                       out);
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
// are the a's, [npair, 2 npair) the b's, and a's item_first / rows_per_item give the
// pair's work items (blocks of rows).  A workgroup stages both owner tables and
// last-dim coordinate tables of its item's pair in LDS when the pair changes, and the
// pair's joint runs along the last dim: maximal stretches of cells whose entries in
// both tables equal their left neighbour's (same owners in every row).  Each wave
// takes every fourth row of the item and works out the row's base index under both
// mappings from the outer tables.  Every cell's two entries are read (a row whose
// entries are all zero has one owner pair), then the runs are evaluated one per lane,
// times their length; a row with the same two base indices as the previous one of the
// wave (the same outer blocks in both) reuses each lane's share.  Rows longer than
// kRedistMaxL cells, or with more than kRedistRuns runs, compare the two owner keys
// of four consecutive cells per lane instead.  Counts go to the pair's totals with
// one atomic per wave and item.

__global__ void k_redist_zero(tm_redist_cost* __restrict__ out, int64_t npair) {
    int64_t* o = reinterpret_cast<int64_t*>(out);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 4 * npair; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = 0;
}

__global__ void k_redist_bytes(tm_redist_cost* __restrict__ out, int64_t npair, int64_t elem_bytes) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npair; i += (int64_t)gridDim.x * blockDim.x) {
        out[i].bytes = out[i].moved_cells * elem_bytes;
        out[i].inter_bytes = out[i].inter_cells * elem_bytes;
    }
}

__global__ __launch_bounds__(256) void k_redist(const DevCand* __restrict__ cands, int64_t npair,
                                                const int32_t* __restrict__ arena, int64_t total_items,
                                                tm_redist_cost* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // 16-byte aligned: ds_read_b128 of the tables
    __shared__ int32_t s_scan[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t cur = -1, rows = 0, ifirst = 0;
    int32_t K = 1, L = 0, gbits = 0, rpi = 1, wa = 0, wb = 0, nrun = 0;
    int32_t offa[TM_MAX_LRANK] = {0, 0, 0, 0}, offb[TM_MAX_LRANK] = {0, 0, 0, 0}, ext[TM_MAX_LRANK] = {1, 1, 1, 1};
    const int32_t *GA = arena, *GB = arena, *CA = lds, *CB = lds;
    // a contiguous range of items per workgroup: consecutive items share a pair, so
    // its tables and runs are staged once per range rather than once per item
    const int64_t per = (total_items + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = i0 + per < total_items ? i0 + per : total_items;
    for (int64_t item = i0; item < i1; ++item) {
        int64_t lo = 0, hi = npair - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (cands[mid].item_first <= item) lo = mid;
            else hi = mid - 1;
        }
        lo = uniform64(lo);
        if (lo != cur) {
            __syncthreads();  // no wave still reads the previous pair's tables
            const DevCand* a = &cands[lo];
            const DevCand* b = &cands[npair + lo];
            const int32_t na = uniform32(a->lds_words), nb = uniform32(b->lds_words);
            wa = (na + 3) & ~3;
            wb = (nb + 3) & ~3;
            GA = arena + uniform64(a->arena_off);
            GB = arena + uniform64(b->arena_off);
            for (int i = tid; i < na; i += 256) lds[i] = GA[i];
            for (int i = tid; i < nb; i += 256) lds[wa + i] = GB[i];
            K = uniform32(a->lrank);
            L = uniform32(a->L);
            gbits = uniform32(a->gbits);
            rpi = uniform32(a->rows_per_item);
            rows = uniform64(a->rows);
            ifirst = uniform64(a->item_first);
            for (int d = 0; d < TM_MAX_LRANK; ++d) {
                offa[d] = uniform32(a->coord_off[d]);
                offb[d] = uniform32(b->coord_off[d]);
                ext[d] = d < K ? uniform32((int32_t)a->extent[d]) : 1;
            }
            CA = uniform32(a->cl_lds) ? lds + offa[K - 1] : GA + offa[K - 1];
            CB = uniform32(b->cl_lds) ? lds + wa + offb[K - 1] : GB + offb[K - 1];
            cur = lo;
            __syncthreads();
            // joint runs of the last dim: each thread counts the run starts of its
            // stretch of cells, a scan places them, then each writes (length << 16) | x
            int32_t* runs = lds + wa + wb;
            nrun = 0;
            if (L <= kRedistMaxL) {
                const int seg = (L + 255) / 256;
                const int x0 = tid * seg, x1 = x0 + seg < L ? x0 + seg : L;
                int c = 0;
                for (int x = x0; x < x1; ++x) c += (x == 0 || CA[x] != CA[x - 1] || CB[x] != CB[x - 1]) ? 1 : 0;
                // exclusive scan over the workgroup: within each wave by shuffles, then
                // the four wave totals
                int v = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(v, o, 64);
                    if (lane >= o) v += t;
                }
                if (lane == 63) s_scan[wid] = v;
                __syncthreads();
                int wbase = 0;
                for (int w = 0; w < wid; ++w) wbase += s_scan[w];
                const int total = s_scan[0] + s_scan[1] + s_scan[2] + s_scan[3];
                __syncthreads();
                if (total <= kRedistRuns) {
                    int pos = wbase + v - c;
                    for (int x = x0; x < x1; ++x) {
                        if (x == 0 || CA[x] != CA[x - 1] || CB[x] != CB[x - 1]) {
                            int y = x + 1;
                            while (y < L && CA[y] == CA[x] && CB[y] == CB[x]) ++y;
                            runs[pos++] = x | ((y - x) << 16);
                        }
                    }
                    nrun = total;
                }
                __syncthreads();
            }
            nrun = uniform32(nrun);
        }
        const int32_t* TA = lds;
        const int32_t* TB = lds + wa;
        const int32_t* runs = lds + wa + wb;
        const int64_t r0 = (item - ifirst) * rpi;
        const int64_t rb = r0 + rpi < rows ? r0 + rpi : rows;
        uint32_t moved = 0, inter = 0;
        int32_t mba = -1, mbb = -1;
        uint32_t mm = 0, mi = 0;
        // base indices of the wave's next 64 rows, one row per lane (loads in parallel)
        int32_t bab = 0, bbb = 0;
        int t = 64;
        for (int64_t r = r0 + wid; r < rb; r += 4) {
            if (t == 64) {
                t = 0;
                const int64_t ri = r + 4 * (int64_t)lane;
                bab = 0;
                bbb = 0;
                if (ri < rb) {
                    uint32_t rr = (uint32_t)ri;  // rows <= 2^30 (checked on the host)
                    for (int d = K - 2; d >= 0; --d) {
                        const uint32_t e = (uint32_t)ext[d];
                        const int32_t q = (int32_t)(rr % e);
                        rr /= e;
                        bab += GA[offa[d] + q] & kValMask;
                        bbb += GB[offb[d] + q] & kValMask;
                    }
                }
            }
            const int32_t ba = __builtin_amdgcn_readlane(bab, t);
            const int32_t bb = __builtin_amdgcn_readlane(bbb, t);
            ++t;
            if (nrun > 0) {
                // every cell's two entries read; all zero: one owner pair for the row
                int32_t any = 0;
                for (int x = 4 * lane; x < L; x += 256) {
                    const i32x4 ea = *reinterpret_cast<const i32x4*>(CA + x);
                    const i32x4 eb = *reinterpret_cast<const i32x4*>(CB + x);
                    any |= ea.x | ea.y | ea.z | ea.w | eb.x | eb.y | eb.z | eb.w;  // zero past L
                }
                if (__ballot(any != 0) == 0ull) {
                    const int32_t ka = TA[ba], kb = TB[bb];
                    if (lane == 0) {
                        moved += ka != kb ? (uint32_t)L : 0u;
                        inter += (ka >> gbits) != (kb >> gbits) ? (uint32_t)L : 0u;
                    }
                    continue;
                }
                if (ba != mba || bb != mbb) {
                    mm = 0;
                    mi = 0;
                    for (int k = lane; k < nrun; k += 64) {
                        const int32_t run = runs[k];
                        const int32_t x = run & 0xffff;
                        const uint32_t len = (uint32_t)run >> 16;
                        const int32_t ka = TA[ba + (CA[x] & kValMask)];
                        const int32_t kb = TB[bb + (CB[x] & kValMask)];
                        mm += ka != kb ? len : 0u;
                        mi += (ka >> gbits) != (kb >> gbits) ? len : 0u;
                    }
                    mba = ba;
                    mbb = bb;
                }
                moved += mm;
                inter += mi;
                continue;
            }
            int32_t pa = -1, pb = -1;
            uint32_t pm = 0, pi = 0;
            for (int x = 4 * lane; x < L; x += 256) {
                // tables are zero-padded to whole 512-entry chunks: x + 3 is in bounds
                const i32x4 ea = *reinterpret_cast<const i32x4*>(CA + x);
                const i32x4 eb = *reinterpret_cast<const i32x4*>(CB + x);
                const int32_t va[4] = {ea.x, ea.y, ea.z, ea.w}, vb[4] = {eb.x, eb.y, eb.z, eb.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (x + j >= L) break;
                    if (va[j] != pa || vb[j] != pb) {
                        const int32_t ka = TA[ba + (va[j] & kValMask)];
                        const int32_t kb = TB[bb + (vb[j] & kValMask)];
                        pm = ka != kb ? 1u : 0u;
                        pi = (ka >> gbits) != (kb >> gbits) ? 1u : 0u;
                        pa = va[j];
                        pb = vb[j];
                    }
                    moved += pm;
                    inter += pi;
                }
            }
        }
        unsigned long long m64 = moved, i64 = inter;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            m64 += __shfl_xor(m64, o, 64);
            i64 += __shfl_xor(i64, o, 64);
        }
        if (lane == 0 && (m64 | i64)) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].moved_cells), m64);
            atomicAdd(reinterpret_cast<unsigned long long*>(&out[cur].inter_cells), i64);
        }
    }
}

hipError_t launch_redist(const DevCand* cands, int64_t npair, const int32_t* arena, int64_t items,
                         int64_t elem_bytes, tm_redist_cost* out, int grid, int lds_words, hipStream_t s) {
    const int64_t zb = (4 * npair + 255) / 256;
    const int zg = zb < 1 ? 1 : (zb > 1024 ? 1024 : (int)zb);
    hipLaunchKernelGGL(k_redist_zero, dim3(zg), dim3(256), 0, s, out, npair);
    if (items > 0)
        hipLaunchKernelGGL(k_redist, dim3(grid), dim3(256), (size_t)lds_words * 4, s, cands, npair, arena, items,
                           out);
    hipLaunchKernelGGL(k_redist_bytes, dim3(zg), dim3(256), 0, s, out, npair, elem_bytes);
    return hipGetLastError();
}

// ------------------------------------------------------------------ matmul tiles
//
// Work block = (candidate, matrix m in {A,B,C}, 16 x 256 consecutive tiles).  A thread
// owns one tile and walks the reduction index (j for A[i,k], i for B[k,j], k for
// C[i,j]), OR-ing the owner's bit into a processor bitmap of W 64-bit words held in
// registers.  Per-processor counts come from wave ballots over the bitmaps; lane p
// of the wave keeps processor (64*w + p)'s count, and one atomic per wave and word
// adds it to the global per-processor totals.

constexpr int kMatmulChunks = 16;  // a work block covers 16 x 256 tiles of one matrix

template <int W>
__global__ __launch_bounds__(256) void k_matmul(const DevCand* __restrict__ cands, int64_t n,
                                                const int32_t* __restrict__ arena,
                                                const int64_t* __restrict__ proc_off,
                                                unsigned long long* __restrict__ per_proc,
                                                const int64_t* __restrict__ block_first, int64_t total_blocks) {
    extern __shared__ __attribute__((aligned(16))) int32_t lds[];  // 16-byte aligned: ds_read_b128 of staged tables
    __shared__ DevCand sc;
    const int lane = threadIdx.x & 63;
    int64_t cur = -1;
    for (int64_t blk = blockIdx.x; blk < total_blocks; blk += gridDim.x) {
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (block_first[mid] <= blk) lo = mid;
            else hi = mid - 1;
        }
        if (lo != cur) {
            __syncthreads();
            stage_cand(&sc, &cands[lo]);
            __syncthreads();
            const int32_t* src = arena + sc.arena_off;
            for (int i = threadIdx.x; i < sc.words; i += blockDim.x) lds[i] = src[i];  // every table
            __syncthreads();
            cur = lo;
        }
        const int64_t Ti = sc.extent[0], Tj = sc.extent[1], Tk = sc.extent[2];
        const int64_t nA = Ti * Tk, nB = Tk * Tj, nC = Ti * Tj;
        const int64_t per = 256 * kMatmulChunks;
        const int64_t bA = (nA + per - 1) / per, bB = (nB + per - 1) / per;
        int64_t local = blk - block_first[lo];
        int m;
        if (local < bA) m = 0;
        else if (local < bA + bB) { m = 1; local -= bA; }
        else { m = 2; local -= bA + bB; }
        const int64_t ntile = m == 0 ? nA : (m == 1 ? nB : nC);
        const int32_t* T = lds;
        const int32_t* C0 = lds + sc.coord_off[0];
        const int32_t* C1 = lds + sc.coord_off[1];
        const int32_t* C2 = lds + sc.coord_off[2];
        const int32_t gb = sc.gbits, g = sc.gpus, gmask = (1 << sc.gbits) - 1;
        uint32_t mine[W];
#pragma unroll
        for (int w = 0; w < W; ++w) mine[w] = 0;
        for (int ch = 0; ch < kMatmulChunks; ++ch) {
            const int64_t tile = (local * kMatmulChunks + ch) * 256 + threadIdx.x;
            if (tile - threadIdx.x >= ntile) break;  // uniform: chunk past the end
            uint64_t bm[W];
#pragma unroll
            for (int w = 0; w < W; ++w) bm[w] = 0;
            if (tile < ntile) {
                int32_t fixed;
                const int32_t* red;
                int64_t nred;
                if (m == 0) {  // A[i,k]: tile = i*Tk + k, reduce over j
                    const int64_t i = tile / Tk, k = tile % Tk;
                    fixed = (C0[i] & kValMask) + (C2[k] & kValMask);
                    red = C1;
                    nred = Tj;
                } else if (m == 1) {  // B[k,j]: tile = k*Tj + j, reduce over i
                    const int64_t k = tile / Tj, j = tile % Tj;
                    fixed = (C2[k] & kValMask) + (C1[j] & kValMask);
                    red = C0;
                    nred = Ti;
                } else {  // C[i,j]: tile = i*Tj + j, reduce over k
                    const int64_t i = tile / Tj, j = tile % Tj;
                    fixed = (C0[i] & kValMask) + (C1[j] & kValMask);
                    red = C2;
                    nred = Tk;
                }
                for (int64_t t = 0; t < nred; ++t) {
                    const int32_t key = T[fixed + (red[t] & kValMask)];
                    const int32_t p = (key >> gb) * g + (key & gmask);
                    const uint64_t bit = 1ull << (p & 63);
                    if (W == 1) {
                        bm[0] |= bit;
                    } else {
#pragma unroll
                        for (int w = 0; w < W; ++w) bm[w] |= ((p >> 6) == w) ? bit : 0ull;
                    }
                }
            }
            // lane b of the wave counts processor 64*w + b
#pragma unroll
            for (int w = 0; w < W; ++w) {
                for (int b = 0; b < 64; ++b) {
                    const uint64_t mask = __ballot((bm[w] >> b) & 1ull);
                    if (lane == b) mine[w] += (uint32_t)__popcll(mask);
                }
            }
        }
        const int64_t P = (int64_t)sc.nodes * sc.gpus;
        unsigned long long* dst = per_proc + proc_off[lo] * 3;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int64_t p = (int64_t)w * 64 + lane;
            if (mine[w] && p < P) atomicAdd(&dst[p * 3 + m], (unsigned long long)mine[w]);
        }
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
                           per_proc, block_first, total_blocks);                                        \
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
