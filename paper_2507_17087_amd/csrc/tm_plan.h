// tm_plan.h -- internal view of batch plans (shared by the plan and search code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "tm_internal.h"

namespace tmk {

// A validated batch: compiled descriptors (host copy) and its sizes.
struct Compiled {
    std::vector<DevCand> cands;
    DevHeader hdr{};
    int64_t arena_words = 0, items = 0, points = 0, max_points = 0;
    int32_t max_words = 0;      // largest LDS-staged prefix
    int32_t max_all_words = 0;  // largest whole table block of one candidate
    int32_t max_vol = 0;        // largest final-space volume
    int32_t cnt_words = 0;      // LDS words of the counting launch (largest staged owner table + class blocks)
    int64_t tuples = 0;         // class-tuple bound of the batch (sum of the candidates')
    int64_t tables_words = 0;   // arena words of the tables (the item table follows)
    int32_t max_citems = 0;     // most counting work items of one candidate
    int K = 0, H = 1;
};

// Device buffers of a search over a loaded plan (grown on demand).
struct SearchBufs {
    int64_t cap_n = 0, cap_sc = 0, cap_pre = 0, cap_sel = 0, cap_seg = 0, cap_words = 0, cap_all = 0;
    uint16_t* X = nullptr;          // [n][kFeat] bf16 features
    float* Y = nullptr;             // [n][kOut] network outputs
    float* score = nullptr;         // [cap_sc] ranking scores (both stages)
    float* cross = nullptr;         // [cap_sc][16] crossing fractions, then [cap_sc][2] fp64 estimates
    int64_t* pre = nullptr;         // [nseg*prefilter] candidates kept by the network's scores
    int64_t* seg = nullptr;         // [nseg+1] instance segments
    int64_t* sel = nullptr;         // [nseg*k] chosen candidate indices
    DevCand* sub = nullptr;         // [nseg*k] survivors
    int64_t* map = nullptr;         // [nseg*k] survivor -> candidate index
    int64_t* sub_seg = nullptr;     // [nseg+1] survivor segments
    DevHeader* sub_hdr = nullptr;
    int32_t* sub_arena = nullptr;
    unsigned long long* sub_counter = nullptr;
    tm_stencil_cost* sub_out = nullptr;
    int64_t* sub_best = nullptr;    // [nseg]
    tm_stencil_cost* all_out = nullptr;  // [n] exhaustive costs
    int64_t nseg = 0, k = 0;
};

}  // namespace tmk

struct tm_plan {
    int device = 0;
    int64_t cap_cands = 0, cap_words = 0;
    tmk::DevCand* d_cands = nullptr;
    int32_t* d_arena = nullptr;
    tmk::DevHeader* d_hdr = nullptr;
    unsigned long long* d_counter = nullptr;
    tmk::DevCand* h_cands = nullptr;  // pinned staging
    tmk::DevHeader* h_hdr = nullptr;
    int64_t* h_seg = nullptr;         // pinned staging for search segments
    int64_t cap_hseg = 0;
    hipEvent_t up_ev = nullptr;
    bool up_pending = false;
    hipStream_t cap_stream = nullptr;
    tmk::Compiled cp;  // the loaded batch
    bool loaded = false;
    int64_t cells_per_item = 0;
    int wg_per_cu = 0;
    // graph cache: one entry
    bool g_valid = false;
    int g_grid = 0;
    void* g_out = nullptr;
    void* g_best = nullptr;
    hipGraphExec_t g_full = nullptr, g_stage[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t g_map = nullptr;  // the whole run, then the map of the selected candidate
    void* g_map_ptr = nullptr;
    tmk::SearchBufs sb;
};

namespace tmk {

// Validates and compiles n candidates on the host (st == nullptr: tables without
// classes; need_lds: every owner table must fit the kernels' LDS budget).
int compile_batch(const tm_candidate* c, int64_t n, const tm_stencil* st, int64_t tuples_per_item, bool need_lds,
                  Compiled& cp);
// Grid of the persistent counting launch for `items` work items.
int count_grid(int lds_words, int64_t items, int wg_per_cu);

int64_t plan_size(const tm_plan* p);
const DevCand* plan_cands(const tm_plan* p);
int32_t plan_max_vol(const tm_plan* p);
const int32_t* plan_halo(const tm_plan* p);
const DevHeader* plan_hdr(const tm_plan* p);
int64_t plan_cells_per_item(const tm_plan* p);
int plan_features(const tm_plan* p, float* d_feat, hipStream_t s);
int plan_block_estimates(const tm_plan* p, double* d_est, hipStream_t s);
int plan_search_prepare(tm_plan* p, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk, bool ranked,
                        SearchBufs** out, hipStream_t s);
hipError_t plan_eval_sub(tm_plan* p, SearchBufs* sb, hipStream_t s);
int plan_exhaustive_search(tm_plan* p, const int64_t* seg, int64_t nseg, int64_t* d_best,
                           tm_stencil_cost* d_best_cost, hipStream_t s);

}  // namespace tmk
