// tm_device.cpp -- device entry points of libtaskmap: single-shot evaluation calls
// and batch plans (persistent counting launch replayed from hipGraphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "tm_internal.h"
#include "tm_plan.h"
#include "tm_ranker.h"

namespace tmk {

#define TM_HIP(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return set_error(TM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Default counting work-item size when the caller gives none: about 16 items per
// CU over the batch's class-tuple bound, between 2^10 and 2^16 tuples.
static int num_cus();
static int64_t default_tuples_per_item(int64_t tuples) {
    const int64_t target = tuples / (int64_t(num_cus()) * 16);
    int64_t c = int64_t(1) << 10;
    while (c < target && c < (int64_t(1) << 16)) c <<= 1;
    return c;
}
// Largest work item accepted from a caller.
constexpr int64_t kMaxCellsPerItem = int64_t(1) << 26;
// Map launches: one workgroup per block of map_rows_per_block(L) rows, up to this many
// (more blocks are taken grid-stride).
constexpr int64_t kMapMaxGrid = int64_t(1) << 20;
static int map_grid(int64_t rows, int32_t L, int32_t lds_words) {
    const int64_t rpb = map_rows_per_block(L, map_narrow(lds_words));
    return (int)std::max<int64_t>(1, std::min<int64_t>((rows + rpb - 1) / rpb, kMapMaxGrid));
}

// ------------------------------------------------------------------ batch compilation

static int64_t up4(int64_t x) { return (x + 3) & ~int64_t(3); }

// Arena layout of one candidate: owner table T, the last dim's coordinate table
// (16-byte aligned, zero-padded to whole 512-entry chunks), the other dims'
// coordinate tables, then (stencil batches: halo != nullptr) the class record (the
// class count of each dim, written by the table build) and each dim's class block
// (entries, starts, offset lists of 2H words; capacities from class_cap).  The map
// and redistribution kernels stage the prefix T + last dim's table in LDS when it
// fits (else T only); the counting kernel stages T and the class blocks.
static int layout_tables(DevCand& d, int H, const int32_t* halo) {
    const int K = d.lrank;
    int64_t off = up4(d.vol);
    const int64_t t_end = off + 4;
    d.coord_off[K - 1] = (int32_t)std::min<int64_t>(off, INT32_MAX);
    off += (d.extent[K - 1] + 511) & ~int64_t(511);  // zero-padded to whole 512-entry chunks
    const int64_t c_end = off + 4;                   // slack for the last four-entry read of a ragged row
    off = std::max(off, c_end);
    for (int k = 0; k < K - 1; ++k) {
        d.coord_off[k] = (int32_t)std::min<int64_t>(off, INT32_MAX);
        off += d.extent[k];
    }
    d.hstride = 2 * H;
    for (int k = 0; k < TM_MAX_LRANK; ++k) d.cls_off[k] = d.cls_cap[k] = 0;
    d.cls_base = d.cls_words = 0;
    if (halo) {
        off = up4(off);
        const int64_t cb = off;
        off += 4;
        for (int k = 0; k < K; ++k) {
            const int64_t cap = class_cap(d, k, halo[k]);
            if (off > INT32_MAX || cap > INT32_MAX / std::max(1, 2 * H)) return TM_EOVERFLOW;
            d.cls_cap[k] = (int32_t)cap;
            d.cls_off[k] = (int32_t)off;
            off += up4(cap) + up4(cap + 1) + up4(cap * 2 * H);
        }
        if (off - cb > INT32_MAX) return TM_EOVERFLOW;
        d.cls_base = (int32_t)cb;
        d.cls_words = (int32_t)(off - cb);
    }
    d.cl_lds = c_end <= kMaxLdsWords ? 1 : 0;
    const int64_t staged = d.cl_lds ? c_end : t_end;
    const int64_t words = up4(std::max(off, staged));  // the next candidate's tables start 16-byte aligned
    if (words > INT32_MAX) return TM_EOVERFLOW;
    d.lds_words = (int32_t)staged;
    d.words = (int32_t)words;
    return TM_OK;
}

// Counting work items of every candidate, and the item table (the candidate of each
// item, written by the table build) after the tables in the arena.
static void layout_items(Compiled& cp, int64_t tuples_per_item) {
    int64_t items = 0;
    cp.max_citems = 0;
    for (auto& d : cp.cands) {
        d.citems = count_items(d, tuples_per_item);
        d.item_first = items;
        items += d.citems;
        cp.max_citems = std::max(cp.max_citems, d.citems);
    }
    cp.items = items;
    cp.hdr.total_items = items;
    cp.hdr.item_tab = cp.tables_words;
    cp.arena_words = cp.tables_words + up4(items);
}

// Validates and compiles n candidates.  st == nullptr: tables without halo flags.
// need_lds: every candidate's tables must fit the LDS budget of the kernels.
int compile_batch(const tm_candidate* c, int64_t n, const tm_stencil* st, int64_t tuples_per_item, bool need_lds,
                  Compiled& cp) {
    if (n < 0) return set_error(TM_EINVAL, "n = %lld", (long long)n);
    if (n > 0 && !c) return set_error(TM_EINVAL, "null candidate array");
    cp.cands.resize((size_t)n);
    cp.hdr = DevHeader{};
    cp.hdr.n = n;
    if (st) {
        if (st->lrank < 1 || st->lrank > TM_MAX_LRANK) return set_error(TM_EINVAL, "stencil lrank %d", st->lrank);
        if (st->elem_bytes < 0) return set_error(TM_EINVAL, "elem_bytes %d", st->elem_bytes);
        int hmax = 0;
        for (int d = 0; d < st->lrank; ++d) {
            if (st->halo[d] < 0 || st->halo[d] > TM_MAX_HALO) return set_error(TM_EINVAL, "halo[%d] = %d", d, st->halo[d]);
            hmax = std::max(hmax, st->halo[d]);
            cp.hdr.halo[d] = st->halo[d];
        }
        if (hmax > kMaxHalo) return set_error(TM_ENOTSUP, "halo %d above the kernels' limit of %d", hmax, kMaxHalo);
        cp.K = 0;  // the largest launch rank in the batch
        cp.H = std::max(1, hmax);
        cp.hdr.elem_bytes = st->elem_bytes;
        cp.hdr.lrank = st->lrank;
        cp.hdr.H = cp.H;
    }
    int64_t words = 0;
    for (int64_t i = 0; i < n; ++i) {
        Shapes sh;
        int rc = validate_shapes(&c[i], &sh);
        if (rc != TM_OK) return set_error(rc, "candidate %lld: %s", (long long)i, tm_last_error());
        // a candidate of launch rank k takes the stencil's first k halo widths
        if (st && c[i].lrank > st->lrank)
            return set_error(TM_EINVAL, "candidate %lld: lrank %d but the stencil has %d", (long long)i, c[i].lrank,
                             st->lrank);
        DevCand& d = cp.cands[(size_t)i];
        rc = fill_devcand(&c[i], sh, &d);
        if (rc == TM_OK) rc = layout_tables(d, st ? cp.H : 0, st ? cp.hdr.halo : nullptr);
        if (rc != TM_OK) return set_error(rc, "candidate %lld: tables too large", (long long)i);
        if (need_lds && d.lds_words > kMaxLdsWords)
            return set_error(TM_ENOTSUP, "candidate %lld: %d table words exceed the LDS budget of %d", (long long)i,
                             d.lds_words, kMaxLdsWords);
        // row indices are 32-bit in the kernels, with room to step past the last row
        if (d.rows > (int64_t(1) << 30))
            return set_error(TM_ENOTSUP, "candidate %lld: more than 2^30 rows", (long long)i);
        d.arena_off = words;
        words += d.words;
        cp.max_words = std::max(cp.max_words, d.lds_words);
        cp.max_all_words = std::max(cp.max_all_words, d.words);
        if (st) {
            const int64_t cw = up4(d.vol) + d.cls_words;  // counting: staged when it fits, else read in place
            if (cw <= kMaxLdsWords) cp.cnt_words = std::max<int32_t>(cp.cnt_words, (int32_t)cw);
            int64_t b = 1;
            for (int k = 0; k < d.lrank; ++k) b = std::min<int64_t>(b * d.cls_cap[k], int64_t(1) << 50);
            cp.tuples += b;
            cp.K = std::max(cp.K, (int)d.lrank);
        }
        cp.points += d.npoints;
        cp.max_points = std::max(cp.max_points, d.npoints);
        cp.max_vol = std::max(cp.max_vol, d.vol);
    }
    cp.tables_words = words;
    cp.arena_words = words;
    cp.hdr.max_words = cp.max_words;
    cp.hdr.cnt_words = cp.cnt_words;
    layout_items(cp, tuples_per_item > 0 ? tuples_per_item : default_tuples_per_item(cp.tuples));
    return TM_OK;
}

// ------------------------------------------------------------------ staging

// Per-thread pinned staging for descriptor uploads; reused once the previous copy
// out of it has completed.
struct Staging {
    void* ptr = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    int device = -1;
    bool pending = false;
};
static thread_local Staging g_stage;

static int staging_acquire(size_t bytes, void** out) {
    int dev = 0;
    TM_HIP(hipGetDevice(&dev));
    if (g_stage.pending) {
        TM_HIP(hipEventSynchronize(g_stage.ev));
        g_stage.pending = false;
    }
    if (g_stage.device != dev) {
        if (g_stage.ev) (void)hipEventDestroy(g_stage.ev);
        g_stage.ev = nullptr;
        g_stage.device = dev;
    }
    if (!g_stage.ev) TM_HIP(hipEventCreateWithFlags(&g_stage.ev, hipEventDisableTiming));
    if (g_stage.cap < bytes) {
        if (g_stage.ptr) TM_HIP(hipHostFree(g_stage.ptr));
        g_stage.ptr = nullptr;
        g_stage.cap = 0;
        const size_t cap = std::max<size_t>(bytes, 1 << 20);
        if (hipHostMalloc(&g_stage.ptr, cap, hipHostMallocDefault) != hipSuccess)
            return set_error(TM_ENOMEM, "pinned staging of %zu bytes", cap);
        g_stage.cap = cap;
    }
    *out = g_stage.ptr;
    return TM_OK;
}

static int staging_release(hipStream_t s) {
    TM_HIP(hipEventRecord(g_stage.ev, s));
    g_stage.pending = true;
    return TM_OK;
}

// Device copies of a compiled batch in stream-ordered allocations.
struct DeviceBatch {
    DevCand* cands = nullptr;
    DevHeader* hdr = nullptr;
    int32_t* arena = nullptr;
    unsigned long long* counter = nullptr;
};

static int upload_batch(const Compiled& cp, DeviceBatch& db, hipStream_t s) {
    const size_t nc = cp.cands.size() * sizeof(DevCand);
    TM_HIP(hipMallocAsync((void**)&db.cands, std::max<size_t>(nc, 64), s));
    TM_HIP(hipMallocAsync((void**)&db.hdr, sizeof(DevHeader) + 64, s));
    TM_HIP(hipMallocAsync((void**)&db.arena, std::max<size_t>((size_t)cp.arena_words * 4, 64), s));
    TM_HIP(hipMallocAsync((void**)&db.counter, 64, s));
    void* stg = nullptr;
    int rc = staging_acquire(nc + sizeof(DevHeader), &stg);
    if (rc != TM_OK) return rc;
    std::memcpy(stg, &cp.hdr, sizeof(DevHeader));
    if (nc) std::memcpy((char*)stg + sizeof(DevHeader), cp.cands.data(), nc);
    TM_HIP(hipMemcpyAsync(db.hdr, stg, sizeof(DevHeader), hipMemcpyHostToDevice, s));
    if (nc) TM_HIP(hipMemcpyAsync(db.cands, (char*)stg + sizeof(DevHeader), nc, hipMemcpyHostToDevice, s));
    return staging_release(s);
}

static void free_batch(DeviceBatch& db, hipStream_t s) {
    if (db.cands) (void)hipFreeAsync(db.cands, s);
    if (db.hdr) (void)hipFreeAsync(db.hdr, s);
    if (db.arena) (void)hipFreeAsync(db.arena, s);
    if (db.counter) (void)hipFreeAsync(db.counter, s);
    db = DeviceBatch{};
}

static int num_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

int count_grid(int lds_words, int64_t items, int wg_per_cu) {
    int per_cu = 0;
    if (count_kernel_occupancy(lds_words, &per_cu) != 0 || per_cu < 1) per_cu = 1;
    if (wg_per_cu > 0) per_cu = std::min(per_cu, wg_per_cu);
    const int64_t g = (int64_t)per_cu * num_cus();
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, items));
}

}  // namespace tmk

using namespace tmk;

// ------------------------------------------------------------------ single-shot calls

extern "C" int tm_chain_table(const tm_candidate* c, int32_t* d_out, int64_t cap, int64_t* count, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    Compiled cp;
    int rc = compile_batch(c, 1, nullptr, 0, false, cp);
    if (rc != TM_OK) return rc;
    if (count) *count = cp.cands[0].vol;
    if (cap < cp.cands[0].vol) return set_error(TM_ECAPACITY, "chain table has %d entries", cp.cands[0].vol);
    if (!d_out) return set_error(TM_EINVAL, "null output");
    DeviceBatch db;
    rc = upload_batch(cp, db, s);
    if (rc == TM_OK) {
        hipError_t e = launch_build_tables(db.hdr, db.cands, 1, db.arena, 0, s);
        if (e == hipSuccess) e = launch_chain_table(db.cands, db.arena, d_out, s);
        if (e != hipSuccess) rc = set_error(TM_EDEVICE, "chain table launch: %s", hipGetErrorString(e));
    }
    free_batch(db, s);
    return rc;
}

extern "C" int tm_proc_map(const tm_candidate* c, int32_t* d_map, int64_t len, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    Compiled cp;
    int rc = compile_batch(c, 1, nullptr, 0, true, cp);
    if (rc != TM_OK) return rc;
    if (len != cp.cands[0].npoints)
        return set_error(TM_ECAPACITY, "map length %lld but the domain has %lld points", (long long)len,
                         (long long)cp.cands[0].npoints);
    if (!d_map) return set_error(TM_EINVAL, "null output");
    DeviceBatch db;
    rc = upload_batch(cp, db, s);
    if (rc == TM_OK) {
        const int grid = map_grid(cp.cands[0].rows, cp.cands[0].L, cp.max_words);
        hipError_t e = launch_build_tables(db.hdr, db.cands, 1, db.arena, 0, s);
        if (e == hipSuccess) e = launch_map(db.cands, 1, db.arena, nullptr, 0, d_map, grid, cp.max_words, s);
        if (e != hipSuccess) rc = set_error(TM_EDEVICE, "map launch: %s", hipGetErrorString(e));
    }
    free_batch(db, s);
    return rc;
}

static int eval_stencil(const tm_candidate* c, int64_t n, const tm_stencil* st, tm_stencil_cost* d_out,
                        hipStream_t s, bool node_level) {
    if (!st) return set_error(TM_EINVAL, "null stencil");
    Compiled cp;
    int rc = compile_batch(c, n, st, 0, true, cp);
    if (rc != TM_OK) return rc;
    cp.hdr.node_level = node_level ? 1 : 0;
    if (n == 0) return TM_OK;
    if (!d_out) return set_error(TM_EINVAL, "null output");
    DeviceBatch db;
    rc = upload_batch(cp, db, s);
    if (rc == TM_OK) {
        const int grid = count_grid(cp.cnt_words, cp.items, 0);
        const bool fin = n <= kFinInCount;
        hipError_t e = launch_build_tables(db.hdr, db.cands, n, db.arena, 1, s, d_out, db.counter);
        if (e == hipSuccess)
            e = launch_count(db.hdr, db.cands, db.arena, db.counter, d_out, grid, cp.cnt_words, s, fin, nullptr);
        if (e == hipSuccess && !fin) e = launch_finalize_select(db.hdr, d_out, nullptr, n, s);
        if (e != hipSuccess) rc = set_error(TM_EDEVICE, "stencil launch: %s", hipGetErrorString(e));
    }
    free_batch(db, s);
    return rc;
}

extern "C" int tm_eval_stencil_batch(const tm_candidate* c, int64_t n, const tm_stencil* st,
                                     tm_stencil_cost* d_out, void* stream) {
    return eval_stencil(c, n, st, d_out, (hipStream_t)stream, false);
}

extern "C" int tm_eval_stencil_node_batch(const tm_candidate* c, int64_t n, const tm_stencil* st,
                                          tm_stencil_cost* d_out, void* stream) {
    return eval_stencil(c, n, st, d_out, (hipStream_t)stream, true);
}

extern "C" int tm_eval_redistribution_batch(const tm_candidate* src, const tm_candidate* dst, int64_t n,
                                            int64_t elem_bytes, tm_redist_cost* d_out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (n < 0) return set_error(TM_EINVAL, "n = %lld", (long long)n);
    if (elem_bytes < 0) return set_error(TM_EINVAL, "elem_bytes %lld", (long long)elem_bytes);
    if (n > 0 && (!src || !dst)) return set_error(TM_EINVAL, "null candidate array");
    for (int64_t i = 0; i < n; ++i) {
        const tm_candidate &a = src[i], &b = dst[i];
        bool same = a.lrank == b.lrank && a.nodes == b.nodes && a.gpus_per_node == b.gpus_per_node;
        for (int d = 0; same && d < a.lrank && d < TM_MAX_LRANK; ++d) same = a.extent[d] == b.extent[d];
        if (!same) return set_error(TM_EINVAL, "pair %lld: different launch domains or machines", (long long)i);
    }
    std::vector<tm_candidate> both((size_t)(2 * n));
    if (n > 0) {
        std::memcpy(both.data(), src, (size_t)n * sizeof(tm_candidate));
        std::memcpy(both.data() + n, dst, (size_t)n * sizeof(tm_candidate));
    }
    Compiled cp;
    int rc = compile_batch(both.data(), 2 * n, nullptr, 0, false, cp);
    if (rc != TM_OK) return rc;
    if (n == 0) return TM_OK;
    if (!d_out) return set_error(TM_EINVAL, "null output");
    // each pair's joint-class block goes into its a-side table block: the record, then
    // per dim the a entries, the b entries and the run starts of its classes; a dim's
    // joint classes start where either mapping's contribution changes, so there are at
    // most 1 + changes_a + changes_b of them.  Work items split the pair's class-tuple
    // bound; the item table follows the tables.
    const int64_t tuples_per_item = int64_t(1) << 12;
    int64_t words = 0, items = 0;
    int32_t lds_words = 0;
    for (int64_t i = 0; i < 2 * n; ++i) {
        DevCand& d = cp.cands[(size_t)i];
        if (i < n) {
            const DevCand& b = cp.cands[(size_t)(n + i)];
            int64_t off = up4(d.words), bound = 1;
            d.cls_base = (int32_t)std::min<int64_t>(off, INT32_MAX);
            off += 4;
            for (int k = 0; k < d.lrank; ++k) {
                const int64_t cap = std::min<int64_t>(d.extent[k], class_cap(d, k, 0) + class_cap(b, k, 0) - 1);
                d.cls_cap[k] = (int32_t)cap;
                d.cls_off[k] = (int32_t)std::min<int64_t>(off, INT32_MAX);
                off += 2 * up4(cap) + up4(cap + 1);
                bound = std::min<int64_t>(bound * cap, int64_t(1) << 50);
            }
            if (off > INT32_MAX) return set_error(TM_EOVERFLOW, "pair %lld: tables too large", (long long)i);
            d.cls_words = (int32_t)(off - d.cls_base);
            d.words = (int32_t)off;
            d.citems = (int32_t)std::min<int64_t>(std::max<int64_t>((bound + tuples_per_item - 1) / tuples_per_item, 1),
                                                  int64_t(1) << 30);
            d.item_first = items;
            items += d.citems;
            const int64_t need = up4(d.vol) + up4(b.vol) + d.cls_words;  // staged when it fits the budget
            if (need <= kMaxLdsWords) lds_words = std::max<int32_t>(lds_words, (int32_t)need);
        }
        d.arena_off = words;
        words += d.words;
    }
    const int64_t item_tab = words;
    cp.arena_words = words + up4(items);
    DeviceBatch db;
    rc = upload_batch(cp, db, s);
    if (rc == TM_OK) {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)num_cus() * 8));
        hipError_t e = launch_build_tables(db.hdr, db.cands, 2 * n, db.arena, 0, s);
        if (e == hipSuccess)
            e = launch_redist(db.cands, n, db.arena, item_tab, items, elem_bytes, d_out, db.counter, grid, lds_words, s);
        if (e != hipSuccess) rc = set_error(TM_EDEVICE, "redistribution launch: %s", hipGetErrorString(e));
    }
    free_batch(db, s);
    return rc;
}

extern "C" int tm_eval_matmul_batch(const tm_candidate* c, int64_t n, const tm_matmul* mm, int64_t* d_per_proc,
                                    tm_matmul_cost* d_out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (!mm || mm->tile_bytes < 0) return set_error(TM_EINVAL, "bad matmul descriptor");
    // coordinate classes with a zero halo: runs of coordinates with equal contributions
    tm_stencil zs{};
    zs.lrank = TM_MAX_LRANK;
    Compiled cp;
    int rc = compile_batch(c, n, &zs, 0, false, cp);
    if (rc != TM_OK) return rc;
    if (n == 0) return TM_OK;
    if (!d_out) return set_error(TM_EINVAL, "null output");
    std::vector<int64_t> proc_off((size_t)n + 1), block_first((size_t)n + 1);
    int64_t procs = 0, blocks = 0;
    int pmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        const DevCand& d = cp.cands[(size_t)i];
        if (d.lrank != 3) return set_error(TM_EINVAL, "candidate %lld: matmul needs launch rank 3", (long long)i);
        const int64_t P = (int64_t)d.nodes * d.gpus;
        if (P > 1024) return set_error(TM_ENOTSUP, "candidate %lld: %lld processors (limit 1024)", (long long)i, (long long)P);
        if (d.extent[0] * d.extent[1] > INT32_MAX || d.extent[1] * d.extent[2] > INT32_MAX ||
            d.extent[0] * d.extent[2] > INT32_MAX)
            return set_error(TM_ENOTSUP, "candidate %lld: more than 2^31 tiles in a matrix", (long long)i);
        pmax = std::max<int>(pmax, (int)P);
        proc_off[(size_t)i] = procs;
        block_first[(size_t)i] = blocks;
        procs += P;
        blocks += matmul_blocks(d);
    }
    proc_off[(size_t)n] = procs;
    block_first[(size_t)n] = blocks;
    DeviceBatch db;
    rc = upload_batch(cp, db, s);
    int64_t *d_off = nullptr, *d_bf = nullptr;
    unsigned long long* d_pp = nullptr;
    if (rc == TM_OK) {
        hipError_t e = hipMallocAsync((void**)&d_off, (size_t)(n + 1) * 8, s);
        if (e == hipSuccess) e = hipMallocAsync((void**)&d_bf, (size_t)(n + 1) * 8, s);
        if (e == hipSuccess) e = hipMallocAsync((void**)&d_pp, (size_t)std::max<int64_t>(procs, 1) * 24, s);
        void* stg = nullptr;
        if (e == hipSuccess) {
            // the descriptor upload above used the staging buffer; reuse waits for it
            rc = staging_acquire((size_t)(n + 1) * 16, &stg);
            if (rc == TM_OK) {
                std::memcpy(stg, proc_off.data(), (size_t)(n + 1) * 8);
                std::memcpy((char*)stg + (n + 1) * 8, block_first.data(), (size_t)(n + 1) * 8);
                e = hipMemcpyAsync(d_off, stg, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(d_bf, (char*)stg + (n + 1) * 8, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s);
                if (e == hipSuccess) rc = staging_release(s);
            }
        }
        if (rc == TM_OK && e == hipSuccess) e = hipMemsetAsync(d_pp, 0, (size_t)std::max<int64_t>(procs, 1) * 24, s);
        if (rc == TM_OK && e == hipSuccess) e = launch_build_tables(db.hdr, db.cands, n, db.arena, 1, s);
        if (rc == TM_OK && e == hipSuccess)
            e = launch_matmul(db.cands, n, db.arena, cp.cnt_words, pmax, d_off, d_pp, blocks, d_bf, s);
        if (rc == TM_OK && e == hipSuccess)
            e = launch_matmul_finalize(db.cands, n, d_off, d_pp, mm->tile_bytes, d_out, d_per_proc, s);
        if (rc == TM_OK && e != hipSuccess) rc = set_error(TM_EDEVICE, "matmul launch: %s", hipGetErrorString(e));
    }
    if (d_off) (void)hipFreeAsync(d_off, s);
    if (d_bf) (void)hipFreeAsync(d_bf, s);
    if (d_pp) (void)hipFreeAsync(d_pp, s);
    free_batch(db, s);
    return rc;
}

extern "C" int tm_select_best(const tm_stencil_cost* d_costs, const int64_t* seg, int64_t nseg, int64_t* d_best,
                              void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (nseg < 0 || (nseg > 0 && (!seg || !d_best))) return set_error(TM_EINVAL, "bad segments");
    if (nseg == 0) return TM_OK;
    for (int64_t i = 0; i < nseg; ++i)
        if (seg[i] < 0 || seg[i + 1] < seg[i]) return set_error(TM_EINVAL, "segment %lld is not ordered", (long long)i);
    if (seg[nseg] > 0 && !d_costs) return set_error(TM_EINVAL, "null costs");
    int64_t* d_seg = nullptr;
    TM_HIP(hipMallocAsync((void**)&d_seg, (size_t)(nseg + 1) * 8, s));
    void* stg = nullptr;
    int rc = staging_acquire((size_t)(nseg + 1) * 8, &stg);
    if (rc == TM_OK) {
        std::memcpy(stg, seg, (size_t)(nseg + 1) * 8);
        hipError_t e = hipMemcpyAsync(d_seg, stg, (size_t)(nseg + 1) * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) rc = staging_release(s);
        if (rc == TM_OK && e == hipSuccess) e = launch_select_segments(d_costs, d_seg, nseg, d_best, s);
        if (rc == TM_OK && e != hipSuccess) rc = set_error(TM_EDEVICE, "select launch: %s", hipGetErrorString(e));
    }
    (void)hipFreeAsync(d_seg, s);
    return rc;
}

// ------------------------------------------------------------------ batch plans

namespace tmk {

static void plan_drop_graphs(tm_plan* p) {
    if (p->g_full) (void)hipGraphExecDestroy(p->g_full);
    if (p->g_map) (void)hipGraphExecDestroy(p->g_map);
    for (auto& g : p->g_stage)
        if (g) (void)hipGraphExecDestroy(g);
    p->g_full = nullptr;
    p->g_map = nullptr;
    p->g_map_ptr = nullptr;
    for (auto& g : p->g_stage) g = nullptr;
    p->g_valid = false;
}

static void search_free(SearchBufs& b) {
    void* ptrs[] = {b.X, b.Y, b.score, b.pre, b.cross, b.seg, b.sel, b.sub, b.map, b.sub_seg, b.sub_hdr,
                    b.sub_arena, b.sub_counter, b.sub_out, b.sub_best, b.all_out};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    b = SearchBufs{};
}

static void plan_free(tm_plan* p) {
    plan_drop_graphs(p);
    search_free(p->sb);
    if (p->d_cands) (void)hipFree(p->d_cands);
    if (p->d_arena) (void)hipFree(p->d_arena);
    if (p->d_hdr) (void)hipFree(p->d_hdr);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->h_cands) (void)hipHostFree(p->h_cands);
    if (p->h_hdr) (void)hipHostFree(p->h_hdr);
    if (p->h_seg) (void)hipHostFree(p->h_seg);
    p->d_cands = nullptr;
    p->d_arena = nullptr;
    p->d_hdr = nullptr;
    p->d_counter = nullptr;
    p->h_cands = nullptr;
    p->h_hdr = nullptr;
    p->h_seg = nullptr;
    p->cap_hseg = 0;
    p->cap_cands = 0;
    p->cap_words = 0;
}

// Descriptor buffers for up to `cands` candidates (the table arena is allocated
// separately, on first use, by plan_ensure_arena).
static int plan_alloc(tm_plan* p, int64_t cands) {
    plan_free(p);
    cands = std::max<int64_t>(cands, 1);
    if (hipMalloc((void**)&p->d_cands, (size_t)cands * sizeof(DevCand)) != hipSuccess ||
        hipMalloc((void**)&p->d_hdr, sizeof(DevHeader)) != hipSuccess ||
        hipMalloc((void**)&p->d_counter, 256) != hipSuccess ||
        hipHostMalloc((void**)&p->h_cands, (size_t)cands * sizeof(DevCand), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&p->h_hdr, sizeof(DevHeader), hipHostMallocDefault) != hipSuccess) {
        plan_free(p);
        return set_error(TM_ENOMEM, "plan buffers for %lld candidates", (long long)cands);
    }
    p->cap_cands = cands;
    return TM_OK;
}

// Table arena of the whole loaded batch; grows (after draining `s`) when needed.
static int plan_ensure_arena(tm_plan* p, hipStream_t s) {
    const int64_t words = std::max<int64_t>(p->cp.arena_words, 1);
    if (p->d_arena && p->cap_words >= words) return TM_OK;
    TM_HIP(hipStreamSynchronize(s));
    if (p->d_arena) (void)hipFree(p->d_arena);
    p->d_arena = nullptr;
    p->cap_words = 0;
    plan_drop_graphs(p);
    if (hipMalloc((void**)&p->d_arena, (size_t)words * 4) != hipSuccess)
        return set_error(TM_ENOMEM, "table arena of %lld words", (long long)words);
    p->cap_words = words;
    return TM_OK;
}

static int plan_upload(tm_plan* p, hipStream_t s) {
    if (p->up_pending) {
        TM_HIP(hipEventSynchronize(p->up_ev));
        p->up_pending = false;
    }
    const size_t nc = p->cp.cands.size() * sizeof(DevCand);
    std::memcpy(p->h_hdr, &p->cp.hdr, sizeof(DevHeader));
    if (nc) std::memcpy(p->h_cands, p->cp.cands.data(), nc);
    TM_HIP(hipMemcpyAsync(p->d_hdr, p->h_hdr, sizeof(DevHeader), hipMemcpyHostToDevice, s));
    if (nc) TM_HIP(hipMemcpyAsync(p->d_cands, p->h_cands, nc, hipMemcpyHostToDevice, s));
    TM_HIP(hipEventRecord(p->up_ev, s));
    p->up_pending = true;
    return TM_OK;
}

// Enqueues one stage of a run on stream s (direct launches; also used for capture).
static hipError_t plan_enqueue(tm_plan* p, int stage, tm_stencil_cost* out, int64_t* best, int grid, hipStream_t s) {
    const Compiled& cp = p->cp;
    const bool fin = cp.hdr.n <= kFinInCount;  // bytes and selection inside the counting launch
    hipError_t e = hipSuccess;
    if (stage == 0 || stage < 0) {
        e = launch_build_tables(p->d_hdr, p->d_cands, cp.hdr.n, p->d_arena, 1, s, out, p->d_counter);
        if (e != hipSuccess) return e;
    }
    if (stage == 1 || stage < 0) {
        e = launch_count(p->d_hdr, p->d_cands, p->d_arena, p->d_counter, out, grid, cp.cnt_words, s, fin, best);
        if (e != hipSuccess) return e;
    }
    // stage 2 on its own repeats the selection (idempotent); the whole run needs it
    // only when the counting launch did not do it
    if (stage == 2 || (stage < 0 && !fin)) e = launch_finalize_select(p->d_hdr, out, best, cp.hdr.n, s);
    return e;
}

static int capture(tm_plan* p, int stage, tm_stencil_cost* out, int64_t* best, int grid, hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    TM_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e = plan_enqueue(p, stage, out, best, grid, p->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(TM_EDEVICE, "capture: %s", hipGetErrorString(e));
    }
    TM_HIP(e2);
    const hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    TM_HIP(e3);
    return TM_OK;
}

// Map grid for a device-side index: the largest over the loaded candidates.
static int plan_map_grid(const tm_plan* p) {
    int grid = 1;
    for (auto& d : p->cp.cands) grid = std::max(grid, map_grid(d.rows, d.L, p->cp.max_words));
    return grid;
}

// The whole run followed by the map of candidate *best, as one graph.
static int capture_run_map(tm_plan* p, tm_stencil_cost* out, int64_t* best, int32_t* map, int grid,
                           hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    TM_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = plan_enqueue(p, -1, out, best, grid, p->cap_stream);
    if (e == hipSuccess)
        e = launch_map(p->d_cands, p->cp.hdr.n, p->d_arena, best, 0, map, plan_map_grid(p), p->cp.max_words,
                       p->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(TM_EDEVICE, "capture: %s", hipGetErrorString(e));
    }
    TM_HIP(e2);
    const hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    TM_HIP(e3);
    return TM_OK;
}

static int plan_graphs(tm_plan* p, tm_stencil_cost* out, int64_t* best) {
    const int grid = count_grid(p->cp.cnt_words, p->cp.items, p->wg_per_cu);
    if (p->g_valid && p->g_grid == grid && p->g_out == out && p->g_best == best) return TM_OK;
    plan_drop_graphs(p);
    int rc = capture(p, -1, out, best, grid, &p->g_full);
    for (int st = 0; st < 3 && rc == TM_OK; ++st) rc = capture(p, st, out, best, grid, &p->g_stage[st]);
    if (rc != TM_OK) {
        plan_drop_graphs(p);
        return rc;
    }
    p->g_valid = true;
    p->g_grid = grid;
    p->g_out = out;
    p->g_best = best;
    return TM_OK;
}

}  // namespace tmk

extern "C" int tm_plan_create(int64_t max_cands, int64_t max_words, tm_plan** out) {
    if (!out) return set_error(TM_EINVAL, "null output");
    *out = nullptr;
    tm_plan* p = new (std::nothrow) tm_plan();
    if (!p) return set_error(TM_ENOMEM, "plan");
    (void)hipGetDevice(&p->device);
    int rc = plan_alloc(p, max_cands);
    if (rc == TM_OK && max_words > 0) {
        if (hipMalloc((void**)&p->d_arena, (size_t)max_words * 4) != hipSuccess) rc = set_error(TM_ENOMEM, "arena");
        else p->cap_words = max_words;
    }
    if (rc == TM_OK && hipEventCreateWithFlags(&p->up_ev, hipEventDisableTiming) != hipSuccess)
        rc = set_error(TM_EDEVICE, "event");
    if (rc == TM_OK && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        rc = set_error(TM_EDEVICE, "capture stream");
    if (rc != TM_OK) {
        tm_plan_destroy(p);
        return rc;
    }
    *out = p;
    return TM_OK;
}

extern "C" int tm_plan_destroy(tm_plan* p) {
    if (!p) return TM_OK;
    if (p->up_pending) (void)hipEventSynchronize(p->up_ev);
    (void)hipDeviceSynchronize();
    plan_free(p);
    if (p->up_ev) (void)hipEventDestroy(p->up_ev);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
    return TM_OK;
}

extern "C" int tm_plan_load(tm_plan* p, const tm_candidate* c, int64_t n, const tm_stencil* st,
                            int64_t cells_per_item, void* stream) {
    if (!p) return set_error(TM_EINVAL, "null plan");
    if (!st) return set_error(TM_EINVAL, "null stencil");
    if (cells_per_item < 0 || cells_per_item > kMaxCellsPerItem)
        return set_error(TM_EINVAL, "cells_per_item %lld (at most 2^26)", (long long)cells_per_item);
    hipStream_t s = (hipStream_t)stream;
    Compiled cp;
    int rc = compile_batch(c, n, st, cells_per_item > 0 ? cells_per_item : p->cells_per_item, true, cp);
    if (rc != TM_OK) return rc;
    if (n > p->cap_cands) {
        // grow: wait for work that may still read the old buffers
        TM_HIP(hipStreamSynchronize(s));
        rc = plan_alloc(p, std::max(n, p->cap_cands));
        if (rc != TM_OK) return rc;
        p->up_pending = false;
    }
    if (cells_per_item > 0) p->cells_per_item = cells_per_item;
    p->cp = std::move(cp);
    p->loaded = true;
    plan_drop_graphs(p);
    return plan_upload(p, s);
}

extern "C" int tm_plan_run(tm_plan* p, tm_stencil_cost* d_out, int64_t* d_best, void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (p->cp.hdr.n > 0 && !d_out) return set_error(TM_EINVAL, "null output");
    if (p->cp.hdr.n == 0) return TM_OK;
    int rc = plan_ensure_arena(p, (hipStream_t)stream);
    if (rc == TM_OK) rc = plan_graphs(p, d_out, d_best);
    if (rc != TM_OK) return rc;
    TM_HIP(hipGraphLaunch(p->g_full, (hipStream_t)stream));
    return TM_OK;
}

extern "C" int tm_plan_run_map(tm_plan* p, tm_stencil_cost* d_out, int64_t* d_best, int32_t* d_map, int64_t cap,
                               void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (p->cp.hdr.n == 0) return set_error(TM_EINVAL, "empty batch");
    if (!d_out || !d_best || !d_map) return set_error(TM_EINVAL, "null output");
    if (cap < p->cp.max_points) return set_error(TM_ECAPACITY, "map needs %lld entries", (long long)p->cp.max_points);
    int rc = plan_ensure_arena(p, (hipStream_t)stream);
    if (rc == TM_OK) rc = plan_graphs(p, d_out, d_best);
    if (rc == TM_OK && (!p->g_map || p->g_map_ptr != d_map)) {
        if (p->g_map) (void)hipGraphExecDestroy(p->g_map);
        p->g_map = nullptr;
        rc = capture_run_map(p, d_out, d_best, d_map, p->g_grid, &p->g_map);
        p->g_map_ptr = rc == TM_OK ? d_map : nullptr;
    }
    if (rc != TM_OK) return rc;
    TM_HIP(hipGraphLaunch(p->g_map, (hipStream_t)stream));
    return TM_OK;
}

extern "C" int tm_plan_run_stage(tm_plan* p, int32_t stage, tm_stencil_cost* d_out, int64_t* d_best,
                                 void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (stage < 0 || stage > 2) return set_error(TM_EINVAL, "stage %d", stage);
    if (p->cp.hdr.n > 0 && !d_out) return set_error(TM_EINVAL, "null output");
    if (p->cp.hdr.n == 0) return TM_OK;
    int rc = plan_ensure_arena(p, (hipStream_t)stream);
    if (rc == TM_OK) rc = plan_graphs(p, d_out, d_best);
    if (rc != TM_OK) return rc;
    TM_HIP(hipGraphLaunch(p->g_stage[stage], (hipStream_t)stream));
    return TM_OK;
}

extern "C" int tm_plan_materialize(tm_plan* p, const int64_t* d_index, int64_t host_index, int32_t* d_map,
                                   int64_t cap, void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (!d_map) return set_error(TM_EINVAL, "null output");
    const Compiled& cp = p->cp;
    if (cp.hdr.n == 0) return set_error(TM_EINVAL, "empty batch");
    int64_t need = cp.max_points;
    int grid = 1;
    if (!d_index) {
        if (host_index < 0 || host_index >= cp.hdr.n) return set_error(TM_EINVAL, "index %lld", (long long)host_index);
        need = cp.cands[(size_t)host_index].npoints;
        grid = map_grid(cp.cands[(size_t)host_index].rows, cp.cands[(size_t)host_index].L, cp.max_words);
    } else {
        grid = plan_map_grid(p);
    }
    if (cap < need) return set_error(TM_ECAPACITY, "map needs %lld entries", (long long)need);
    if (!p->d_arena || p->cap_words < cp.arena_words)
        return set_error(TM_EINVAL, "no tables yet: run the plan before materialising a map");
    const hipError_t e = launch_map(p->d_cands, cp.hdr.n, p->d_arena, d_index, host_index, d_map, grid, cp.max_words,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "map launch: %s", hipGetErrorString(e));
    return TM_OK;
}

extern "C" int tm_plan_info(const tm_plan* p, int64_t* n, int64_t* items, int64_t* points) {
    if (!p) return set_error(TM_EINVAL, "null plan");
    if (n) *n = p->loaded ? p->cp.hdr.n : 0;
    if (items) *items = p->loaded ? p->cp.items : 0;
    if (points) *points = p->loaded ? p->cp.points : 0;
    return TM_OK;
}

extern "C" int tm_plan_class_tuples(tm_plan* p, int64_t* tuples, void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (!tuples) return set_error(TM_EINVAL, "null output");
    *tuples = 0;
    if (p->cp.hdr.n == 0) return TM_OK;
    if (!p->d_arena || p->cap_words < p->cp.arena_words) return set_error(TM_EINVAL, "no tables yet: run the plan first");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d_tot = nullptr;
    TM_HIP(hipMallocAsync((void**)&d_tot, 8, s));
    unsigned long long h = 0;
    hipError_t e = hipMemsetAsync(d_tot, 0, 8, s);
    if (e == hipSuccess) e = launch_class_tuples(p->d_cands, p->cp.hdr.n, p->d_arena, d_tot, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d_tot, 8, hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(d_tot, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "class tuples: %s", hipGetErrorString(e));
    *tuples = (int64_t)h;
    return TM_OK;
}

extern "C" int tm_plan_autotune(tm_plan* p, tm_stencil_cost* d_out, int64_t* cells_per_item, int32_t* wg_per_cu,
                                void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (p->cp.hdr.n == 0) return TM_OK;
    if (!d_out) return set_error(TM_EINVAL, "null output");
    hipStream_t s = (hipStream_t)stream;
    int arc = plan_ensure_arena(p, s);
    if (arc != TM_OK) return arc;
    hipEvent_t e0, e1;
    TM_HIP(hipEventCreate(&e0));
    TM_HIP(hipEventCreate(&e1));
    const int64_t cells_opts[] = {1 << 10, 1 << 12, 1 << 14};
    const int wg_opts[] = {0, 2, 1};
    float best_ms = 1e30f;
    int64_t best_c = default_tuples_per_item(p->cp.tuples);
    int best_w = 0;
    int rc = TM_OK;
    for (int64_t cpi : cells_opts) {
        layout_items(p->cp, cpi);
        rc = plan_ensure_arena(p, s);
        if (rc == TM_OK) rc = plan_upload(p, s);
        if (rc != TM_OK) break;
        // tables once per layout (they do not depend on it)
        if (plan_enqueue(p, 0, d_out, nullptr, 1, s) != hipSuccess) {
            rc = set_error(TM_EDEVICE, "autotune build");
            break;
        }
        for (int w : wg_opts) {
            const int grid = count_grid(p->cp.cnt_words, p->cp.items, w);
            float tot = 0.f;
            for (int rep = 0; rep < 3 && rc == TM_OK; ++rep) {
                hipError_t e = launch_reset(p->d_hdr, p->d_counter, d_out, p->cp.hdr.n, s);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                if (e == hipSuccess) e = plan_enqueue(p, 1, d_out, nullptr, grid, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) rc = set_error(TM_EDEVICE, "autotune: %s", hipGetErrorString(e));
                if (rep > 0) tot += ms;
            }
            if (rc != TM_OK) break;
            if (tot < best_ms) {
                best_ms = tot;
                best_c = cpi;
                best_w = w;
            }
        }
        if (rc != TM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TM_OK) return rc;
    p->cells_per_item = best_c;
    p->wg_per_cu = best_w;
    layout_items(p->cp, best_c);
    plan_drop_graphs(p);
    rc = plan_ensure_arena(p, s);
    if (rc == TM_OK) rc = plan_upload(p, s);
    if (cells_per_item) *cells_per_item = best_c;
    if (wg_per_cu) *wg_per_cu = best_w;
    return rc;
}

extern "C" int tm_plan_set_launch(tm_plan* p, int64_t cells_per_item, int32_t wg_per_cu, void* stream) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (cells_per_item < 0 || cells_per_item > kMaxCellsPerItem || wg_per_cu < 0)
        return set_error(TM_EINVAL, "cells_per_item %lld (at most 2^26), wg_per_cu %d", (long long)cells_per_item,
                         wg_per_cu);
    p->cells_per_item = cells_per_item;
    p->wg_per_cu = wg_per_cu;
    if (p->cp.hdr.n == 0) return TM_OK;
    layout_items(p->cp, cells_per_item > 0 ? cells_per_item : default_tuples_per_item(p->cp.tuples));
    plan_drop_graphs(p);
    return plan_upload(p, (hipStream_t)stream);
}

// ------------------------------------------------------------------ search support

namespace tmk {

int64_t plan_size(const tm_plan* p) { return p->cp.hdr.n; }
const DevCand* plan_cands(const tm_plan* p) { return p->d_cands; }
int32_t plan_max_vol(const tm_plan* p) { return p->cp.max_vol; }
const int32_t* plan_halo(const tm_plan* p) { return p->d_hdr->halo; }
const DevHeader* plan_hdr(const tm_plan* p) { return p->d_hdr; }
int64_t plan_cells_per_item(const tm_plan* p) {
    return p->cells_per_item > 0 ? p->cells_per_item : default_tuples_per_item(p->cp.tuples);
}

// Ranker buffers: features and outputs of n rows; scores and chain statistics of
// max(n, m) entries (m: the second stage's survivors of a ranked search).
static int ensure_rank_bufs(SearchBufs& b, int64_t n, int64_t m, hipStream_t s) {
    const int64_t sc = std::max<int64_t>(std::max(n, m), 1);
    if (b.cap_n < n) {
        TM_HIP(hipStreamSynchronize(s));
        if (b.X) (void)hipFree(b.X);
        if (b.Y) (void)hipFree(b.Y);
        b.X = nullptr;
        b.Y = nullptr;
        b.cap_n = 0;
        if (hipMalloc((void**)&b.X, (size_t)std::max<int64_t>(n, 1) * kFeat * 2) != hipSuccess ||
            hipMalloc((void**)&b.Y, (size_t)std::max<int64_t>(n, 1) * kOut * 4) != hipSuccess)
            return set_error(TM_ENOMEM, "feature buffers");
        b.cap_n = n;
    }
    if (b.cap_sc < sc) {
        TM_HIP(hipStreamSynchronize(s));
        if (b.score) (void)hipFree(b.score);
        if (b.cross) (void)hipFree(b.cross);
        b.score = b.cross = nullptr;
        b.cap_sc = 0;
        if (hipMalloc((void**)&b.score, (size_t)sc * 4) != hipSuccess ||
            hipMalloc((void**)&b.cross, (size_t)sc * (kCrossFloats + 4) * 4) != hipSuccess)
            return set_error(TM_ENOMEM, "score buffers");
        b.cap_sc = sc;
    }
    return TM_OK;
}

int plan_features(const tm_plan* p, float* d_feat, hipStream_t s) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (!d_feat) return set_error(TM_EINVAL, "null output");
    tm_plan* q = const_cast<tm_plan*>(p);
    SearchBufs& b = q->sb;
    const int64_t n = p->cp.hdr.n;
    const int rc = ensure_rank_bufs(b, n, 0, s);
    if (rc != TM_OK) return rc;
    TM_HIP(launch_features(p->d_cands, n, p->d_hdr->halo, chain_estimates(b.cross, n), b.X, d_feat, s));
    return TM_OK;
}

int plan_block_estimates(const tm_plan* p, double* d_est, hipStream_t s) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (!d_est) return set_error(TM_EINVAL, "null output");
    tm_plan* q = const_cast<tm_plan*>(p);
    SearchBufs& b = q->sb;
    const int64_t n = p->cp.hdr.n;
    const int rc = ensure_rank_bufs(b, n, 0, s);
    if (rc != TM_OK) return rc;
    TM_HIP(launch_chain_stats(p->d_cands, nullptr, n, p->cp.max_vol, p->d_hdr->halo, b.cross, s));
    if (n > 0)
        TM_HIP(hipMemcpyAsync(d_est, chain_estimates(b.cross, n), (size_t)n * 2 * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    return TM_OK;
}

int plan_search_prepare(tm_plan* p, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk, bool ranked,
                        SearchBufs** out, hipStream_t s) {
    if (!p || !p->loaded) return set_error(TM_EINVAL, "plan not loaded");
    if (nseg < 1 || !seg) return set_error(TM_EINVAL, "no segments");
    const int64_t n = p->cp.hdr.n;
    if (seg[0] != 0 || seg[nseg] != n) return set_error(TM_EINVAL, "segments must cover the loaded batch");
    for (int64_t i = 0; i < nseg; ++i) {
        if (seg[i + 1] < seg[i]) return set_error(TM_EINVAL, "segment %lld is not ordered", (long long)i);
        if (seg[i + 1] - seg[i] > INT32_MAX) return set_error(TM_EINVAL, "segment %lld is too long", (long long)i);
    }
    if (ranked && (topk < 1 || topk > 4096)) return set_error(TM_EINVAL, "topk %d not in 1..4096", topk);
    if (ranked && prefilter != 0 && (prefilter < topk || prefilter > 65536))
        return set_error(TM_EINVAL, "prefilter %d not 0 or in topk..65536", prefilter);
    SearchBufs& b = p->sb;
    const int64_t nsel = ranked ? nseg * (int64_t)topk : 0;
    const int64_t npre = ranked ? nseg * (int64_t)prefilter : 0;
    // survivors' tables, then their item table
    const int64_t words = nsel * (std::max<int64_t>(p->cp.max_all_words, 1) + p->cp.max_citems) + 4;
    auto grow = [&](bool need) -> int {
        if (!need) return TM_OK;
        TM_HIP(hipStreamSynchronize(s));
        return TM_OK;
    };
    if (ranked) {
        int rc = ensure_rank_bufs(b, n, npre, s);
        if (rc != TM_OK) return rc;
        if (b.cap_pre < npre) {
            TM_HIP(hipStreamSynchronize(s));
            if (b.pre) (void)hipFree(b.pre);
            b.pre = nullptr;
            b.cap_pre = 0;
            if (hipMalloc((void**)&b.pre, (size_t)npre * 8) != hipSuccess)
                return set_error(TM_ENOMEM, "prefilter buffer");
            b.cap_pre = npre;
        }
        if (b.cap_sel < nsel || b.cap_words < words) {
            int rc = grow(true);
            if (rc != TM_OK) return rc;
            void* ptrs[] = {b.sel, b.sub, b.map, b.sub_arena, b.sub_out};
            for (void* q : ptrs)
                if (q) (void)hipFree(q);
            b.sel = nullptr;
            b.sub = nullptr;
            b.map = nullptr;
            b.sub_arena = nullptr;
            b.sub_out = nullptr;
            b.cap_sel = b.cap_words = 0;
            if (hipMalloc((void**)&b.sel, (size_t)nsel * 8) != hipSuccess ||
                hipMalloc((void**)&b.sub, (size_t)nsel * sizeof(DevCand)) != hipSuccess ||
                hipMalloc((void**)&b.map, (size_t)nsel * 8) != hipSuccess ||
                hipMalloc((void**)&b.sub_arena, (size_t)std::max<int64_t>(words, 1) * 4) != hipSuccess ||
                hipMalloc((void**)&b.sub_out, (size_t)nsel * sizeof(tm_stencil_cost)) != hipSuccess)
                return set_error(TM_ENOMEM, "survivor buffers");
            b.cap_sel = nsel;
            b.cap_words = words;
        }
        if (!b.sub_hdr) {
            if (hipMalloc((void**)&b.sub_hdr, sizeof(DevHeader)) != hipSuccess ||
                hipMalloc((void**)&b.sub_counter, 256) != hipSuccess)
                return set_error(TM_ENOMEM, "survivor header");
        }
    } else if (b.cap_all < n) {
        int rc = grow(b.all_out != nullptr);
        if (rc != TM_OK) return rc;
        if (b.all_out) (void)hipFree(b.all_out);
        b.all_out = nullptr;
        b.cap_all = 0;
        if (hipMalloc((void**)&b.all_out, (size_t)std::max<int64_t>(n, 1) * sizeof(tm_stencil_cost)) != hipSuccess)
            return set_error(TM_ENOMEM, "cost buffer");
        b.cap_all = n;
    }
    if (b.cap_seg < nseg + 1) {
        int rc = grow(true);
        if (rc != TM_OK) return rc;
        if (b.seg) (void)hipFree(b.seg);
        if (b.sub_seg) (void)hipFree(b.sub_seg);
        if (b.sub_best) (void)hipFree(b.sub_best);
        b.seg = b.sub_seg = b.sub_best = nullptr;
        b.cap_seg = 0;
        if (hipMalloc((void**)&b.seg, (size_t)(nseg + 1) * 8) != hipSuccess ||
            hipMalloc((void**)&b.sub_seg, (size_t)(nseg + 1) * 8) != hipSuccess ||
            hipMalloc((void**)&b.sub_best, (size_t)(nseg + 1) * 8) != hipSuccess)
            return set_error(TM_ENOMEM, "segment buffers");
        b.cap_seg = nseg + 1;
    }
    // segments: copy only when they changed (pinned staging, ordered on s)
    if (b.nseg != nseg || !p->h_seg || std::memcmp(p->h_seg, seg, (size_t)(nseg + 1) * 8) != 0) {
        if (p->up_pending) {
            TM_HIP(hipEventSynchronize(p->up_ev));
            p->up_pending = false;
        }
        if (p->cap_hseg < nseg + 1) {
            if (p->h_seg) (void)hipHostFree(p->h_seg);
            p->h_seg = nullptr;
            if (hipHostMalloc((void**)&p->h_seg, (size_t)(nseg + 1) * 8, hipHostMallocDefault) != hipSuccess)
                return set_error(TM_ENOMEM, "segment staging");
            p->cap_hseg = nseg + 1;
        }
        std::memcpy(p->h_seg, seg, (size_t)(nseg + 1) * 8);
        TM_HIP(hipMemcpyAsync(b.seg, p->h_seg, (size_t)(nseg + 1) * 8, hipMemcpyHostToDevice, s));
        TM_HIP(hipEventRecord(p->up_ev, s));
        p->up_pending = true;
    }
    b.nseg = nseg;
    b.k = topk;
    *out = &b;
    return TM_OK;
}

// Exact costs of the survivors gathered in sb (descriptors and header on device).
hipError_t plan_eval_sub(tm_plan* p, SearchBufs* sb, hipStream_t s) {
    const int64_t nsel = sb->nseg * sb->k;
    const Compiled& cp = p->cp;
    hipError_t e = launch_build_tables(sb->sub_hdr, sb->sub, nsel, sb->sub_arena, 1, s, sb->sub_out, sb->sub_counter);
    if (e == hipSuccess) {
        // survivors' work items are bounded by the batch's largest candidate (its item
        // count under the plan's current layout)
        const int64_t max_items = cp.max_citems;
        const int grid = count_grid(cp.cnt_words, std::max<int64_t>(1, max_items * nsel), p->wg_per_cu);
        e = launch_count(sb->sub_hdr, sb->sub, sb->sub_arena, sb->sub_counter, sb->sub_out, grid, cp.cnt_words, s,
                         nsel <= kFinInCount, nullptr);
    }
    if (e == hipSuccess && nsel > kFinInCount) e = launch_finalize_select(sb->sub_hdr, sb->sub_out, nullptr, nsel, s);
    return e;
}

int plan_exhaustive_search(tm_plan* p, const int64_t* seg, int64_t nseg, int64_t* d_best,
                           tm_stencil_cost* d_best_cost, hipStream_t s) {
    if (!d_best) return set_error(TM_EINVAL, "null output");
    SearchBufs* sb = nullptr;
    int rc = plan_search_prepare(p, seg, nseg, 0, 0, false, &sb, s);
    if (rc == TM_OK) rc = plan_ensure_arena(p, s);
    if (rc != TM_OK) return rc;
    const int grid = count_grid(p->cp.cnt_words, p->cp.items, p->wg_per_cu);
    hipError_t e = plan_enqueue(p, -1, sb->all_out, nullptr, grid, s);
    if (e == hipSuccess) e = launch_select_segments(sb->all_out, sb->seg, nseg, d_best, s);
    if (e == hipSuccess) e = launch_pick_costs(d_best, sb->seg, sb->all_out, nseg, d_best_cost, s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "exhaustive search: %s", hipGetErrorString(e));
    return TM_OK;
}

}  // namespace tmk
