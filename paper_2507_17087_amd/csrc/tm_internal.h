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
    int32_t rows_per_item, L;           // rows per work item; row length = last extent
    int32_t coord_off[TM_MAX_LRANK];    // table offsets of the per-dim coordinate tables
    int32_t dl_off[TM_MAX_LRANK];       // table offsets of the per-dim neighbour-offset lists
    int32_t lds_words, hstride;         // leading words staged in LDS; list stride (2*H)
    int32_t dl_lds, cl_lds;             // last dim's offset lists / coordinate table are in the staged prefix
    int32_t fshape[TM_MAX_MRANK], fstride[TM_MAX_MRANK];
    int8_t proj_src[TM_MAX_MRANK], proj_mode[TM_MAX_MRANK];
    int32_t rank[TM_MAX_OPS];                    // rank before op t
    int32_t shape[TM_MAX_OPS][TM_MAX_MRANK];     // shape before op t
    int32_t op_kind[TM_MAX_OPS], op_a[TM_MAX_OPS], op_b[TM_MAX_OPS], op_nf[TM_MAX_OPS];
    int32_t op_f[TM_MAX_OPS][TM_MAX_LRANK];
};

// Batch header: one per plan, in device memory, read by every kernel of a replay.
struct DevHeader {
    int64_t n;            // candidates
    int64_t total_items;  // work items over all candidates
    int32_t halo[TM_MAX_LRANK];
    int32_t elem_bytes, lrank;
    int32_t max_words, H;  // largest staged table; max halo (0: no neighbour lists)
    int32_t node_level;    // owner tables hold nodes only (node-level exchange volume)
    int32_t pad0;
};

// Host-side result of validation.
struct Shapes {
    int32_t rank[TM_MAX_OPS + 1];
    int64_t size[TM_MAX_OPS + 1][TM_MAX_MRANK];
};

// Word layout of an entry of a per-dim coordinate table: bits 0..23 hold the
// contribution of that coordinate to the linear final-space index (volumes are at
// most 2^24), bits 24..27 the number of distinct non-zero index offsets from that
// coordinate to its star neighbours along the dim (within the halo).  That list of
// offsets is stored separately, 2*H words per coordinate, zero-padded.
constexpr int32_t kValMask = 0x00ffffff;
constexpr int kCntShift = 24;
// Bit 28 of a last-dim entry with offsets: cell x - 1 has the same contribution and
// the same offset list, so (in the same row) the same foreign owners.
constexpr int kSameShift = 28;
// Bit 29: cells x - 1 and x each have a single offset, pointing at the other's
// coordinate (the two sides of one block boundary compare the same pair of owners),
// so in a row without outer offsets both count the same foreign owners.
constexpr int kMirrorShift = 29;
constexpr int32_t kMaxLdsWords = 32768;
// Redistribution: LDS words for the joint runs of a pair's last dim (rows of at most
// kRedistMaxL cells), staged after the pair's two tables.
constexpr int32_t kRedistRuns = 512;
constexpr int32_t kRedistMaxL = 4096;
constexpr int kMaxHalo = 4;

int set_error(int code, const char* fmt, ...);
int validate_shapes(const tm_candidate* c, Shapes* sh);
int fill_devcand(const tm_candidate* c, const Shapes& sh, DevCand* d);

// Kernel launchers (tm_kernels.hip).  All enqueue on `s` and return hipError_t.
hipError_t launch_build_tables(const DevHeader* hdr, const DevCand* cands, int64_t n, int32_t* arena,
                               int32_t mode_halo, hipStream_t s);
hipError_t launch_reset(DevHeader* hdr, unsigned long long* counter, tm_stencil_cost* out, int64_t n,
                        hipStream_t s);
hipError_t launch_count(int K, int H, const DevHeader* hdr, const DevCand* cands, const int32_t* arena,
                        unsigned long long* counter, tm_stencil_cost* out, int grid, int lds_words,
                        hipStream_t s);
hipError_t launch_finalize_select(const DevHeader* hdr, tm_stencil_cost* out, int64_t* best,
                                  hipStream_t s);
hipError_t launch_select_segments(const tm_stencil_cost* costs, const int64_t* seg, int64_t nseg,
                                  int64_t* best, hipStream_t s, const int64_t* key = nullptr);
hipError_t launch_map(const DevCand* cands, int64_t n, const int32_t* arena, const int64_t* d_index,
                      int64_t index, int32_t* out, int grid, int lds_words, hipStream_t s);
hipError_t launch_chain_table(const DevCand* cand, const int32_t* arena, int32_t* out, hipStream_t s);
hipError_t launch_redist(const DevCand* cands, int64_t npair, const int32_t* arena, int64_t items,
                         int64_t elem_bytes, tm_redist_cost* out, int grid, int lds_words, hipStream_t s);
hipError_t launch_matmul(const DevCand* cands, int64_t n, const int32_t* arena, int words_max,
                         int pmax, const int64_t* proc_off, unsigned long long* per_proc,
                         int64_t total_blocks, const int64_t* block_first, hipStream_t s);
hipError_t launch_matmul_finalize(const DevCand* cands, int64_t n, const int64_t* proc_off,
                                  const unsigned long long* per_proc, int64_t tile_bytes,
                                  tm_matmul_cost* out, int64_t* out_per_proc, hipStream_t s);
int count_kernel_occupancy(int K, int H, int lds_words, int* blocks_per_cu);

}  // namespace tmk
