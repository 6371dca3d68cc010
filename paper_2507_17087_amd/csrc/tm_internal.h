// tm_internal.h -- structures shared by the host side and the kernels of libtaskmap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "taskmap.h"

namespace tmk {

// Compiled candidate as the kernels read it.  The host fills in the shapes of the
// processor space before every transformation (validation computes them anyway);
// the table-build kernel derives everything per coordinate from these.
struct DevCand {
    int32_t lrank, nops, nodes, gpus;
    int32_t gbits, frank, vol, words;   // gpu bits of the owner key; final rank and volume; table words
    int64_t extent[TM_MAX_LRANK];
    int64_t npoints;
    int64_t arena_off;                  // word offset of this candidate's tables
    int64_t item_first;                 // first work item of this candidate
    int64_t rows;                       // points / extent[lrank-1]
    int32_t L, pad1;                    // row length = last extent
    int32_t coord_off[TM_MAX_LRANK];    // table offsets of the per-dim coordinate tables
    int32_t cls_off[TM_MAX_LRANK];      // table offsets of the per-dim coordinate-class blocks
    int32_t cls_cap[TM_MAX_LRANK];      // class capacity of each dim (an upper bound on the class count)
    int32_t cls_base, cls_words;        // class record (four class counts) + the blocks: offset and words
    int32_t lds_words, hstride;         // leading words staged in LDS by the map kernel; offset-list stride (2*H)
    int32_t citems, cl_lds;             // counting work items; last dim's coordinate table is in the staged prefix
    int32_t fshape[TM_MAX_MRANK], fstride[TM_MAX_MRANK];
    int8_t proj_src[TM_MAX_MRANK], proj_mode[TM_MAX_MRANK];
    int32_t rank[TM_MAX_OPS];                    // rank before op t
    int32_t shape[TM_MAX_OPS][TM_MAX_MRANK];     // shape before op t
    int32_t op_kind[TM_MAX_OPS], op_a[TM_MAX_OPS], op_b[TM_MAX_OPS], op_nf[TM_MAX_OPS];
    int32_t op_f[TM_MAX_OPS][TM_MAX_LRANK];
    // Inverse of op t on linear indices: the dims the op touches form a contiguous
    // range of its input shape (swap and merge: from the lower to the higher
    // position; the others: one dim), inside which the op maps the range's digits;
    // the dims before and after the range pass through.  inv_lo: product of the
    // input dims after the range; inv_win / inv_wout: volume of the range in the
    // input / output shape; inv_mid: product of the dims strictly inside a swap or
    // merge range; inv_c: the second output extent of a split or balance_split.
    int32_t inv_lo[TM_MAX_OPS], inv_win[TM_MAX_OPS], inv_wout[TM_MAX_OPS], inv_mid[TM_MAX_OPS],
        inv_c[TM_MAX_OPS];
};

// Batch header: one per plan, in device memory, read by every kernel of a replay.
struct DevHeader {
    int64_t n;            // candidates
    int64_t total_items;  // work items over all candidates
    int32_t halo[TM_MAX_LRANK];
    int32_t elem_bytes, lrank;
    int32_t max_words, H;  // largest table prefix staged by the map kernel; max halo (offset-list stride 2H)
    int32_t node_level;    // owner tables hold nodes only (node-level exchange volume)
    int32_t cnt_words;     // LDS words of the counting launch (owner table + class blocks staged)
    int64_t item_tab;      // arena word offset of the item table (candidate of every counting work item)
};

// Host-side result of validation.
struct Shapes {
    int32_t rank[TM_MAX_OPS + 1];
    int64_t size[TM_MAX_OPS + 1][TM_MAX_MRANK];
};

// An entry of a per-dim coordinate table holds the contribution of that coordinate
// to the linear final-space index (volumes are at most 2^24).
//
// Coordinate classes (stencil batches).  Along launch dim d, coordinate x has a
// contribution C_d[x] and a set of distinct non-zero index offsets C_d[x +- s] -
// C_d[x] to its in-domain star neighbours (1 <= s <= h_d).  The distinct foreign
// owners of a cell depend on nothing else: cells whose coordinates fall in the same
// class along every dim have equal counts.  A class is a maximal run of consecutive
// coordinates with equal contribution and equal offset set; its block stores, for
// class k, the entry (contribution | offset count << kCntShift), the first
// coordinate (k = R is the extent, so the run length is start[k+1] - start[k]) and
// the sorted offsets (2*H words, zero-padded).
constexpr int32_t kValMask = 0x00ffffff;
constexpr int kCntShift = 24;
constexpr int32_t kMaxLdsWords = 32768;
constexpr int kMaxHalo = 4;

// Upper bound on the class count of launch dim d (its block capacity): a class
// boundary at x needs a change of contribution within the halo of x (at some c with
// x - h <= c <= x + h), so there are at most 1 + changes * (2h + 1) classes, and
// never more than the extent.  Block projections change at most s - 1 times along
// the dim, cyclic ones at every step.
__host__ __device__ inline int64_t class_cap(const DevCand& c, int d, int h) {
    const int64_t l = c.extent[d];
    int64_t ch = 0;
    for (int j = 0; j < c.frank; ++j) {
        if (c.proj_src[j] != d) continue;
        const int64_t s = c.fshape[j];
        ch += c.proj_mode[j] == TM_BLOCK ? (s - 1 < l - 1 ? s - 1 : l - 1) : l - 1;
    }
    if (ch > l - 1) ch = l - 1;
    const int64_t r = 1 + ch * (2 * (int64_t)h + 1);
    return r < l ? r : l;
}

// Map kernel: when the staged tables are small (many workgroups fit a CU), one-wave
// workgroups taking blocks of about 1,024 points (4 KB of int32 map); else four-wave
// workgroups taking about 4,096 points (16 KB).
constexpr int32_t kMapMaxRowsPerBlock = 64;
constexpr int32_t kMapNarrowWords = 2048;
__host__ __device__ inline bool map_narrow(int32_t lds_words) { return lds_words <= kMapNarrowWords; }
__host__ __device__ inline int32_t map_rows_per_block(int32_t L, bool narrow) {
    const int32_t pts = narrow ? 1024 : 4096;
    const int32_t r = (pts + (L > 0 ? L : 1) - 1) / (L > 0 ? L : 1);
    return r < 1 ? 1 : (r > kMapMaxRowsPerBlock ? kMapMaxRowsPerBlock : r);
}

// Counting work items of a candidate: its class-tuple bound (product of the
// capacities) split into items of about `per_item` tuples (at least one item).
__host__ __device__ inline int32_t count_items(const DevCand& c, int64_t per_item) {
    int64_t b = 1;
    for (int d = 0; d < c.lrank; ++d) {
        b *= c.cls_cap[d] > 0 ? c.cls_cap[d] : 1;
        if (b > (int64_t(1) << 50)) b = int64_t(1) << 50;
    }
    if (per_item < 1) per_item = 1;
    const int64_t it = (b + per_item - 1) / per_item;
    return (int32_t)(it < 1 ? 1 : (it > (int64_t(1) << 30) ? (int64_t(1) << 30) : it));
}

int set_error(int code, const char* fmt, ...);
int validate_shapes(const tm_candidate* c, Shapes* sh);
int fill_devcand(const tm_candidate* c, const Shapes& sh, DevCand* d);

// Kernel launchers (tm_kernels.hip).  All enqueue on `s` and return hipError_t.
// Table build; with out/counter (stencil batches) it also zeroes the outputs and the
// counting kernel's work and completion counters (counter[0], counter[1]).
hipError_t launch_build_tables(const DevHeader* hdr, const DevCand* cands, int64_t n, int32_t* arena,
                               int32_t mode_halo, hipStream_t s, tm_stencil_cost* out = nullptr,
                               unsigned long long* counter = nullptr);
hipError_t launch_reset(DevHeader* hdr, unsigned long long* counter, tm_stencil_cost* out, int64_t n,
                        hipStream_t s);
// Counting; with fin the last workgroup to finish also writes the bytes and, when
// best is given, selects (the work of k_finalize_select; for small batches).
hipError_t launch_count(const DevHeader* hdr, const DevCand* cands, const int32_t* arena,
                        unsigned long long* counter, tm_stencil_cost* out, int grid, int lds_words,
                        hipStream_t s, bool fin = false, int64_t* best = nullptr);
// Batches up to this many candidates finalise inside the counting launch.
constexpr int64_t kFinInCount = 2048;
hipError_t launch_class_tuples(const DevCand* cands, int64_t n, const int32_t* arena, unsigned long long* total,
                               hipStream_t s);
// n_max: an upper bound on the header's candidate count; without best, batches above
// kFinBytesGrid candidates take their bytes in a grid-wide launch.
constexpr int64_t kFinBytesGrid = 65536;
hipError_t launch_finalize_select(const DevHeader* hdr, tm_stencil_cost* out, int64_t* best, int64_t n_max,
                                  hipStream_t s);
hipError_t launch_select_segments(const tm_stencil_cost* costs, const int64_t* seg, int64_t nseg,
                                  int64_t* best, hipStream_t s, const int64_t* key = nullptr);
hipError_t launch_map(const DevCand* cands, int64_t n, const int32_t* arena, const int64_t* d_index,
                      int64_t index, int32_t* out, int grid, int lds_words, hipStream_t s);
hipError_t launch_chain_table(const DevCand* cand, const int32_t* arena, int32_t* out, hipStream_t s);
// Batches of at least this many candidates run the per-candidate table and
// statistics kernels with one-wave workgroups (more candidates in flight per CU).
constexpr int64_t kSmallBlockBatch = 8192;
// Batches of at most this many candidates build their tables with one workgroup per
// (candidate, launch dim) instead of one per candidate.
constexpr int64_t kSplitBuildBatch = 1024;

// Matmul work blocks: kMatmulTiles class pairs of one matrix each.  A matrix over
// launch dims (a, b) has cls_cap[a] * cls_cap[b] class pairs at most; A = (0, 2),
// B = (2, 1), C = (0, 1).
constexpr int kMatmulTiles = 4096;
__host__ __device__ inline int64_t matmul_pair_blocks(int64_t ca, int64_t cb) {
    return (ca * cb + kMatmulTiles - 1) / kMatmulTiles;
}
__host__ __device__ inline int64_t matmul_blocks(const DevCand& d) {
    return matmul_pair_blocks(d.cls_cap[0], d.cls_cap[2]) + matmul_pair_blocks(d.cls_cap[2], d.cls_cap[1]) +
           matmul_pair_blocks(d.cls_cap[0], d.cls_cap[1]);
}

// Redistribution of npair pairs (joint classes, then counting over a work queue,
// then bytes); the arena holds both mappings' tables and each pair's class block.
hipError_t launch_redist(const DevCand* cands, int64_t npair, int32_t* arena, int64_t item_tab, int64_t items,
                         int64_t elem_bytes, tm_redist_cost* out, unsigned long long* counter, int grid,
                         int lds_words, hipStream_t s);
hipError_t launch_matmul(const DevCand* cands, int64_t n, const int32_t* arena, int words_max,
                         int pmax, const int64_t* proc_off, unsigned long long* per_proc,
                         int64_t total_blocks, const int64_t* block_first, hipStream_t s);
hipError_t launch_matmul_finalize(const DevCand* cands, int64_t n, const int64_t* proc_off,
                                  const unsigned long long* per_proc, int64_t tile_bytes,
                                  tm_matmul_cost* out, int64_t* out_per_proc, hipStream_t s);
int count_kernel_occupancy(int lds_words, int* blocks_per_cu);

}  // namespace tmk
