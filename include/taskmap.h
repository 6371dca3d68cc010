/*
 * taskmap.h -- C ABI of libtaskmap: exact, batched evaluation of index-task
 * mappings on an AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Mapple, arXiv 2507.17087, Sec. 3): an index launch has a task
 * space (launch domain) of k dimensions; the machine is the processor space
 * Machine(GPU) = (nodes, GPUs per node) (Sec. 3.2.1).  A mapping transforms the
 * processor space with a chain of primitives -- split, merge, swap (Sec. 3.3,
 * Fig. 6), decompose (Sec. 4.2) and balance_split (named in the paper's listings,
 * never defined; reading below) -- and projects every launch point onto the final
 * space, by blocks (Fig. 1 / Fig. 3: point * size / space) or round robin
 * (Fig. 4).  The processor of a point is found by inverting the chain, last
 * transformation first (Sec. 5.2).  The library returns the processor of every
 * point and the communication the mapping induces:
 *   - stencil ghost volume: for every cell, the distinct processors that own one of
 *     its star neighbours (halo width h_m along dim m) other than its own owner,
 *     split into intra- and inter-node transfers (Sec. 4.1, Sec. 4.2 volume model,
 *     App. A.3 anisotropic halos);
 *   - matmul tile fetches: distinct A[i,k], B[k,j], C[i,j] tiles per processor for a
 *     task space (i,j,k) (the matmul mappers of Sec. 6 and App. A.1);
 *   - redistribution volume between two mappings, e.g. the all-to-all transposes of
 *     App. A.3 (cells whose owner, or owner's node, changes);
 *   - decompose's search (Sec. 4.3): every ordered factorization, the exact argmin
 *     of the objective, the greedy grid of Alg. A1, and a learned ranker that
 *     prunes candidate lists before exact evaluation.
 *
 * Readings where the paper is silent:
 *   - balance_split(i,d) on a dim of size s: shape (.., d, ceil(s/d), ..); the
 *     inverse folds v = a_i + a_{i+1}*d onto b_i = floor(v*s / (d*ceil(s/d))).
 *     Equal to split(i,d) when d divides s; processor loads differ by at most one.
 *   - decompose(i,F) = split(i,F0), split(i+1,F1), ..., so F0 varies fastest.
 *   - processor id = node * gpus_per_node + gpu.
 *   - ghost volume counts distinct (receiving processor, cell) pairs; the domain is
 *     not periodic; a transfer is inter-node when the receiver's node differs from
 *     the node owning the cell.
 *   - all integer division is floor division of non-negative values.
 *
 * Conventions
 *   - Every entry point returns TM_OK (0) or a negative TM_E* code; the message of
 *     the last failure on the calling thread is returned by tm_last_error().
 *   - Validation is complete before anything is enqueued: on error nothing is
 *     launched and no output is touched.
 *   - "host" pointers are read before the call returns; "device" pointers are
 *     caller-owned device memory (e.g. torch tensors) of the current HIP device and
 *     are written by work enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream).  Results are valid once the stream reaches that work.
 *   - Opaque handles (tm_plan, tm_ranker) are created and destroyed only here.
 *   - Calls on different streams are independent; one handle must not be used by
 *     two threads at once.
 */
#ifndef TASKMAP_H
#define TASKMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TM_ABI_VERSION 1

enum { TM_MAX_LRANK = 4, TM_MAX_MRANK = 8, TM_MAX_OPS = 8 };
/* Largest processor-space volume (product of its shape) after any transformation. */
#define TM_MAX_VOLUME (1LL << 24)
#define TM_MAX_EXTENT 2147483647LL
#define TM_MAX_POINTS (1LL << 40)
#define TM_MAX_HALO 65535

enum tm_status {
    TM_OK = 0,
    TM_EINVAL = -1,    /* malformed descriptor or argument */
    TM_EOVERFLOW = -2, /* a size exceeds the documented limits */
    TM_ECAPACITY = -3, /* output buffer too small; *count holds the size needed */
    TM_ENOMEM = -4,    /* host or device allocation failed */
    TM_EDEVICE = -5,   /* a HIP call failed (message in tm_last_error) */
    TM_ENOTSUP = -6    /* valid input outside what the GPU kernels handle */
};

enum tm_op_kind { TM_SPLIT = 1, TM_MERGE = 2, TM_SWAP = 3, TM_BALANCE_SPLIT = 4, TM_DECOMPOSE = 5 };
enum tm_proj_mode { TM_BLOCK = 0, TM_CYCLIC = 1 };

/* One transformation of the processor space (Fig. 6, Sec. 4.2).
 *   split(i=a, d=b)        (.., s_i, ..) -> (.., d, s_i/d, ..); requires d | s_i
 *   merge(p=a, q=b)        p < q; dims p, q fused at p (p fastest), q removed
 *   swap(p=a, q=b)         p != q; the two dims exchanged
 *   balance_split(i=a,d=b) (.., s_i, ..) -> (.., d, ceil(s_i/d), ..)
 *   decompose(i=a, f[0..nf)) s_i replaced by f[0..nf); product of f must be s_i */
typedef struct {
    int32_t kind, a, b, nf;
    int32_t f[TM_MAX_LRANK];
} tm_op;

/* A candidate mapping: 328 bytes, little-endian, 8-byte aligned.
 *   lrank        launch rank k, 1..4
 *   nodes, gpus_per_node  Machine(GPU) = (nodes, gpus_per_node); product <= 2^24
 *   nops         number of transformations applied to Machine(GPU), 0..8
 *   extent[d]    launch domain 0 <= ip[d] < extent[d]; points in C order (last dim
 *                fastest); product <= 2^40
 *   mrank        rank of the final processor space (checked)
 *   proj_src[j]  launch dim projected onto final dim j
 *   proj_mode[j] TM_BLOCK: a_j = floor(ip[src]*s_j / extent[src]);
 *                TM_CYCLIC: a_j = ip[src] mod s_j  */
typedef struct {
    int32_t lrank, nodes, gpus_per_node, nops;
    int64_t extent[TM_MAX_LRANK];
    tm_op ops[TM_MAX_OPS];
    int32_t mrank, reserved;
    int8_t proj_src[TM_MAX_MRANK];
    int8_t proj_mode[TM_MAX_MRANK];
} tm_candidate;

/* Star stencil, non-periodic: halo[d] cells along each axis (0..65535), elements of
 * elem_bytes bytes.  lrank must be at least every candidate's launch rank; a
 * candidate of launch rank k takes halo[0..k), so one batch may mix launch ranks. */
typedef struct {
    int32_t lrank, elem_bytes;
    int32_t halo[TM_MAX_LRANK];
} tm_stencil;

/* ghost_cells = sum over cells of the distinct other owners of a star neighbour;
 * inter_cells = the part whose receiver is on another node; bytes = cells * elem_bytes. */
typedef struct {
    int64_t ghost_cells, inter_cells, bytes, inter_bytes;
} tm_stencil_cost;

/* moved_cells = cells whose owner differs between two mappings; inter_cells = the
 * part whose owner's node differs; bytes = cells * elem_bytes. */
typedef struct {
    int64_t moved_cells, inter_cells, bytes, inter_bytes;
} tm_redist_cost;

/* Matmul task space (i,j,k) = extent[0..2]; each task touches A[i,k], B[k,j], C[i,j]. */
typedef struct {
    int64_t tile_bytes;
} tm_matmul;

/* tiles[m]: sum over processors of distinct tiles of matrix m (A, B, C);
 * max_tiles[m]: largest per-processor count; bytes = sum(tiles) * tile_bytes. */
typedef struct {
    int64_t tiles[3], max_tiles[3], bytes;
} tm_matmul_cost;

int tm_abi_version(void);
int tm_candidate_size(void); /* sizeof(tm_candidate) */
/* Message of the last failed call on this thread ("" if none). */
const char* tm_last_error(void);

/* ---------------------------------------------------------------- host calls */

/* Checks one candidate (host).  On TM_OK writes the final shape (up to 8 entries)
 * and its rank.  Errors: TM_EINVAL (bad kind, index, factor, projection or rank),
 * TM_EOVERFLOW (size limits). */
int tm_validate(const tm_candidate* c, int32_t* final_shape, int32_t* final_rank);

/* decompose's search space (Sec. 4.3): all ordered k-tuples (1 <= k <= 4) of
 * positive integers with product P (1 <= P <= 2^24), lexicographic ascending,
 * written row-major to out[count][k] (host).  *count always receives the number of
 * tuples; TM_ECAPACITY if it exceeds cap (out may be NULL when cap == 0). */
int tm_enumerate_factorizations(int64_t P, int32_t k, int32_t* out, int64_t cap, int64_t* count);

/* decompose's choice (Sec. 4.2, App. A.3): the factorization F of P minimising
 * sum_m halo[m] * F[m] * prod_{j != m} extent[j], compared exactly; ties go to the
 * lexicographically smallest F (host). */
int tm_decompose_argmin(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo,
                        int32_t* out_f);

/* decompose with transposes (App. A.3): the same search, objective
 * sum_m halo[m] F[m] prod_{j != m} extent[j] + sum_{n in T} (1 - 1/F[n]) prod_m extent[m],
 * T = the dims whose bit is set in transpose_mask (an all-to-all along dim n moves
 * all but 1/F[n] of every partition's data); compared exactly, ties to the
 * lexicographically smallest F.  halo[m] <= 255 here (TM_EINVAL beyond), at most
 * 2^40 points (host). */
int tm_decompose_argmin_transpose(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo,
                                  int32_t transpose_mask, int32_t* out_f);

/* The pencil-transposed image of mapping c for an all-to-all transpose along launch
 * dim `dim` (App. A.3: each partition keeps 1/d of its data and sends the rest to the
 * other d - 1 processors of its pencil along `dim`).  Reading: the d processors that
 * share every final coordinate except the one projected from `dim` split their joint
 * data along launch dim `into` instead, d ways inside each block of `into`, with
 * `dim` whole.  Built as c's chain followed by swap (when needed) and merge of the
 * final dim projected from `dim` (the fast part) into the final dim projected from
 * `into`, which is then projected by blocks from `into`; `dim` is no longer
 * projected.  Requires dim != into, exactly one final dim projected from each, both
 * TM_BLOCK, and room for the one or two added ops (TM_EINVAL otherwise).  The
 * transpose's traffic is tm_eval_redistribution_batch(c, *out); with divisible
 * blocks it is (1 - 1/d) * (points) cells, App. A.3's closed form (host). */
int tm_transpose_target(const tm_candidate* c, int32_t dim, int32_t into, tm_candidate* out);

/* Alg. A1 (App. A.2): primes of P ascending, each multiplied into the smallest
 * current factor (lowest index on ties), result sorted descending (host). */
int tm_greedy_grid(int64_t P, int32_t k, int32_t* out_f);

/* The workload greedy of Sec. 4.3: primes ascending, each to the dimension that
 * minimises max(w) - min(w), w_m = extent[m] / F[m], exactly (host). */
int tm_workload_greedy(int64_t P, int32_t k, const int64_t* extent, int32_t* out_f);

/* ---------------------------------------------------------------- device calls */

/* The chain table (Fig. 6's formulas applied last transformation first, as the
 * translator of Sec. 5.2 inverts a mapping): processor id of every coordinate of the
 * final space of c (C order), computed on the GPU: d_out (device, int32[cap]).
 * *count (host) receives the volume; TM_ECAPACITY if cap is smaller. */
int tm_chain_table(const tm_candidate* c, int32_t* d_out, int64_t cap, int64_t* count,
                   void* stream);

/* The processor map (Sec. 3.2.1's index-task mapping; Fig. 3 works one point): the
 * processor id of every launch point of c, C order: d_map (device, int32[len]), len
 * must equal the number of points (else TM_ECAPACITY). */
int tm_proc_map(const tm_candidate* c, int32_t* d_map, int64_t len, void* stream);

/* Stencil cost of n candidates (host array) sharing one stencil (host); results to
 * d_out (device, tm_stencil_cost[n]).  Candidates may differ in launch rank (each
 * at most st->lrank; TM_EINVAL otherwise).  Counted exactly as a weighted sum over
 * coordinate classes: along each launch dim, consecutive coordinates with the same
 * contribution to the final index and the same offsets to their star neighbours
 * form a class, and every cell of a tuple of classes has the same distinct foreign
 * owners (Sec. 4.2's volume, evaluated once per class tuple and multiplied by the
 * cells it stands for).  TM_ENOTSUP if a halo exceeds 4, a candidate's owner table
 * (its final-space volume) exceeds the per-workgroup LDS budget of 32768 words, or
 * it has more than 2^30 rows (points / last extent); the coordinate tables and
 * classes have no size limit (large ones are read from global memory). */
int tm_eval_stencil_batch(const tm_candidate* c, int64_t n, const tm_stencil* st,
                          tm_stencil_cost* d_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): tm_eval_stencil_batch
 * with the same arguments, results and validation, allocating no device memory and
 * no pinned host memory.
 * The batch header, descriptors, tables and work counter live in a device array of
 * TM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends; TM_ECAPACITY (nothing launched) when the batch needs more.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on other
 * streams or threads) race, and the caller must serialise them.  The descriptors are
 * copied from host memory before the call returns (it waits for `stream` to finish
 * those copies, and so for the work enqueued before them); the counting itself runs
 * asynchronously on `stream`. */
#define TM_NOALLOC_SCRATCH_BYTES (64 << 20)
int tm_eval_stencil_batch_noalloc(const tm_candidate* c, int64_t n, const tm_stencil* st,
                                  tm_stencil_cost* d_out, void* stream);

/* Node-level exchange volume (two-level mappings, where a node receives each remote
 * cell once however many of its GPUs read it; App. A.1's hierarchical mappers):
 * for every cell, the distinct nodes other than its owner's node that own one of
 * its star neighbours.  Same arguments, limits and output layout as
 * tm_eval_stencil_batch, with ghost_cells = inter_cells = that count. */
int tm_eval_stencil_node_batch(const tm_candidate* c, int64_t n, const tm_stencil* st,
                               tm_stencil_cost* d_out, void* stream);

/* Redistribution volume of n pairs (src[i], dst[i]) of mappings of the same launch
 * domain on the same Machine(GPU) (host arrays): the cells whose owner under src
 * differs from their owner under dst -- the data a change of mapping moves, e.g. a
 * transpose by all-to-all exchanges (App. A.3; dst from tm_transpose_target) -- and
 * the part whose owner's node changes.  d_out (device, tm_redist_cost[n]).  Counted
 * exactly over joint coordinate classes: along each launch dim, consecutive
 * coordinates with the same contributions under both mappings form a class, and the
 * cells of a tuple of classes all move or all stay.  TM_EINVAL if a pair differs in
 * launch rank, extents or machine (validation messages number src[i] as candidate i
 * and dst[i] as candidate n + i).  Owner tables and classes have no size limit
 * (those that do not fit the LDS budget together are read from global memory). */
int tm_eval_redistribution_batch(const tm_candidate* src, const tm_candidate* dst, int64_t n, int64_t elem_bytes,
                                 tm_redist_cost* d_out, void* stream);

/* Matmul tile fetches (the data movement App. A.1's matmul mappers -- Cannon, SUMMA,
 * Johnson's 3-D, Solomonik's 2.5-D -- differ in) of n rank-3 candidates:
 * d_per_proc (device, int64[sum P_c][3],
 * candidates back to back, may be NULL) and d_out (device, tm_matmul_cost[n]).
 * Counted over coordinate classes: along each launch dim, consecutive coordinates
 * with the same contribution to the final index form a class; all tiles of one pair
 * of classes have the same owner set along the reduction dim, so each owner of the
 * pair counts its tiles at once.  TM_ENOTSUP if a candidate has more than 1024
 * processors or a matrix has more than 2^31 tiles. */
int tm_eval_matmul_batch(const tm_candidate* c, int64_t n, const tm_matmul* mm,
                         int64_t* d_per_proc, tm_matmul_cost* d_out, void* stream);

/* Selection by Sec. 4.2's objective, the communication volume (ties broken by
 * inter-node bytes, then index), over a cost array (device): for each of nseg segments
 * [seg[s], seg[s+1]) of d_costs (seg is a host int64[nseg+1]), the index (relative to
 * the segment start) minimising (bytes, inter_bytes, index) -> d_best (device,
 * int64[nseg]).  Empty segments give -1. */
int tm_select_best(const tm_stencil_cost* d_costs, const int64_t* seg, int64_t nseg,
                   int64_t* d_best, void* stream);

/* ---------------------------------------------------------------- front end
 * Translates the IndexTaskMap mapper of `task` in a mapping-language program (the
 * syntax figure of Sec. 7; Fig. 1 and App. A.1 give examples) into one candidate
 * for the launch domain extent[0..lrank) on Machine(GPU) = (nodes, gpus_per_node).
 * Supported inside the mapper: `def f(Task t)` with t.ipoint / t.ispace, or
 * `def f(Tuple point, Tuple space)`; assignments; integer and element-wise tuple
 * arithmetic (+ - * / // %), tuple literals, indexing, slicing and * unpacking;
 * Machine(GPU) and its methods split / merge / swap / balance_split /
 * decompose(i, domain) (factors from decompose's argmin over `domain`, weighted by
 * `halo` when the domain has the launch rank; halo may be NULL = all 1), .size, and
 * m[i] as the size of dim i inside arithmetic; `return m[...]` whose coordinates are
 * ip[d]*s/ispace[d] (BLOCK) or ip[d]%s (CYCLIC) with s the size of that processor
 * dim, or 0 for a dim of size 1.  Module-level assignments (e.g. m = Machine(GPU))
 * are visible in functions; other statements (Task, Region, Layout, collection
 * and backpressure directives) are ignored.  `IndexTaskMap * f` applies to every
 * task without its own mapper.  Host only, synchronous.  TM_EINVAL with the line
 * and column of the first unsupported construct in tm_last_error(). */
int tm_parse_index_task_map(const char* source, const char* task, int32_t lrank, const int64_t* extent,
                            int32_t nodes, int32_t gpus_per_node, const int32_t* halo, tm_candidate* out);

/* ---------------------------------------------------------------- batch plans
 * A plan owns device memory for up to max_cands candidates and max_words table
 * words.  tm_plan_load validates a batch on the host and uploads its descriptors
 * (asynchronously, on `stream`); tm_plan_run replays one hipGraph: reset -> table
 * build (owner tables, coordinate tables, coordinate classes) -> one persistent
 * counting launch over a work queue of (candidate, range of class tuples) items,
 * whatever the candidates' launch ranks -> bytes + selection.  d_out:
 * tm_stencil_cost[n]; d_best: int64[1] (may be NULL).  Work items hold about
 * cells_per_item class tuples of the candidate's bound (0 = a default from the
 * batch: about 16 items per CU, 2^10 to 2^16 tuples; at most 2^26, else
 * TM_EINVAL). */
typedef struct tm_plan tm_plan;

int tm_plan_create(int64_t max_cands, int64_t max_words, tm_plan** out);
int tm_plan_load(tm_plan* p, const tm_candidate* c, int64_t n, const tm_stencil* st,
                 int64_t cells_per_item, void* stream);
int tm_plan_run(tm_plan* p, tm_stencil_cost* d_out, int64_t* d_best, void* stream);
/* stage 0: table build (which also zeroes d_out and the work counters); 1: counting
 * (for batches of at most 2048 candidates its last workgroup also writes the bytes
 * and selects); 2: bytes + selection (same work as tm_plan_run, one stage at a time,
 * in this order, each replayed from its own graph). */
int tm_plan_run_stage(tm_plan* p, int32_t stage, tm_stencil_cost* d_out, int64_t* d_best,
                      void* stream);
/* Processor map of candidate *d_index (device int64; index into the loaded batch),
 * or of host_index when d_index is NULL, into d_map (device int32[cap]); cap must
 * hold the largest candidate of the batch. */
int tm_plan_materialize(tm_plan* p, const int64_t* d_index, int64_t host_index, int32_t* d_map,
                        int64_t cap, void* stream);
/* tm_plan_run, then the processor map of the selected candidate (*d_best) into
 * d_map (device int32[cap], cap holding the batch's largest candidate), replayed as
 * one hipGraph: Sec. 4.2's choice and the map Sec. 3.2 defines for it, with no host
 * step between them.  d_out, d_best and d_map must not be NULL (TM_EINVAL); an empty
 * batch is TM_EINVAL, a short map TM_ECAPACITY. */
int tm_plan_run_map(tm_plan* p, tm_stencil_cost* d_out, int64_t* d_best, int32_t* d_map, int64_t cap,
                    void* stream);
/* Class tuples of the loaded batch (the counting kernel's work): the sum over its
 * candidates of the product of their per-dim class counts, as built by the last
 * run -> *tuples (host).  Synchronous: waits for `stream`.  TM_EINVAL before the
 * first run. */
int tm_plan_class_tuples(tm_plan* p, int64_t* tuples, void* stream);
/* Times cells_per_item and grid variants of the loaded batch, keeps the fastest;
 * writes the chosen cells_per_item and workgroups per CU (host pointers, nullable). */
int tm_plan_autotune(tm_plan* p, tm_stencil_cost* d_out, int64_t* cells_per_item,
                     int32_t* wg_per_cu, void* stream);
/* Sets the launch configuration of the loaded batch without timing anything: work
 * items of cells_per_item cells (0 = default) and at most wg_per_cu counting
 * workgroups per CU (0 = as many as occupancy allows) -- e.g. a configuration found
 * by tm_plan_autotune earlier.  TM_EINVAL on negative values or cells_per_item above
 * 2^26. */
int tm_plan_set_launch(tm_plan* p, int64_t cells_per_item, int32_t wg_per_cu, void* stream);
/* Counts of the loaded batch: candidates, work items, total points (host, nullable). */
int tm_plan_info(const tm_plan* p, int64_t* n, int64_t* items, int64_t* points);
int tm_plan_destroy(tm_plan* p);

/* ---------------------------------------------------------------- learned ranker
 * A surrogate of the exact cost that prunes decompose's candidate space before
 * exact evaluation (the search of Sec. 4.3 over factorizations, widened to
 * transformation chains).  Model: 64 features -> 3 hidden layers of width 256
 * (ReLU) -> 2 outputs, BF16 weights and activations with FP32 accumulation on the
 * matrix cores, FP32 master weights trained with Adam on the mean squared error
 * against standardised residuals: log2(1 + bytes) and log2(1 + inter-node bytes)
 * of exact costs, each minus the base the features carry (32 * feature 23 and
 * 32 * feature 60, in fp32).  The features come from the descriptor alone (shapes,
 * factors, op kinds and arguments; no pass over the processor space); feature 23
 * is the descriptor estimate of the ghost cells -- along each launch dim, 2h cells
 * of every cross-section at each boundary where the projected final coordinates
 * change (l - 1 of them under a cyclic projection, else the interior block starts),
 * exact for bijective chains whose blocks are at least h wide -- and feature 60 is
 * 0.  Parameters are one flat fp32 vector of tm_ranker_param_count() values:
 * W1[64][256], b1[256], W2[256][256], b2, W3[256][256], b3, W4[256][2], b4[2]
 * (row-major, inputs along rows). */
typedef struct tm_ranker tm_ranker;

int tm_ranker_param_count(void);
int tm_ranker_feature_count(void);
/* He-normal initial weights from `seed`, zero biases. */
int tm_ranker_create(uint64_t seed, tm_ranker** out);
int tm_ranker_destroy(tm_ranker* r);
/* Copies of the fp32 parameter vector (device pointers, param_count floats). */
int tm_ranker_get_params(tm_ranker* r, float* d_out, void* stream);
int tm_ranker_set_params(tm_ranker* r, const float* d_in, void* stream);
/* mu_sigma (host, 4 floats) = {mu0, sigma0, mu1, sigma1} of the target scaling. */
int tm_ranker_get_scaling(const tm_ranker* r, float* mu_sigma);
/* Features of every candidate loaded in plan p (device fp32 [n][64]). */
int tm_ranker_features(const tm_plan* p, float* d_feat, void* stream);
/* Block-model estimates of every candidate loaded in plan p, as tm_search's second
 * stage computes them: d_est (device fp64 [n][2]) = ghost cells, inter-node ghost
 * cells (0, 0 for a processor space above 16384 coordinates). */
int tm_ranker_block_estimates(const tm_plan* p, double* d_est, void* stream);
/* Network outputs for n feature rows (device fp32 [n][64] -> [n][2]); inputs are
 * rounded to bf16 first. */
int tm_ranker_forward(tm_ranker* r, const float* d_feat, int64_t n, float* d_out, void* stream);
/* Gradient of the mean squared error over n rows and both outputs against
 * d_target (device fp32 [n][2], already standardised) -> d_grad (device fp32
 * [param_count]); parameters are not changed. */
int tm_ranker_grad(tm_ranker* r, const float* d_feat, const float* d_target, int64_t n, float* d_grad, void* stream);
/* Trains on n rows: features d_feat (device fp32 [n][64]) and exact costs d_cost
 * (device tm_stencil_cost[n]); sets the target scaling from the data; `epochs`
 * passes in shuffled minibatches of `batch` rows, Adam with cosine-decayed lr.
 * h_loss (host, nullable, [epochs]) receives the loss of each epoch's first batch.
 * Synchronous with respect to the host. */
int tm_ranker_train(tm_ranker* r, const float* d_feat, const tm_stencil_cost* d_cost, int64_t n, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, float* h_loss, void* stream);
int tm_ranker_save(const tm_ranker* r, const char* path);
int tm_ranker_load(const char* path, tm_ranker** out);

/* Search over the batch loaded in plan p, split into nseg instances by seg (host
 * int64[nseg+1], seg[0] = 0, seg[nseg] = n, each at most 2^31 - 1 long).  For each
 * instance, d_best (device int64[nseg]) receives the index (relative to the
 * instance) of the candidate minimising (bytes, inter_bytes, index) and d_best_cost
 * (device, nullable) its cost.  r == NULL: every candidate is evaluated exactly.
 * Otherwise the ranker scores every candidate by predicted log2(1 + bytes) + lambda
 * * predicted log2(1 + inter-node bytes) (base + residual head) and:
 *   prefilter == 0: the topk lowest (score, index) per instance are evaluated
 *     exactly;
 *   prefilter in topk..65536: the prefilter lowest per instance are kept, their
 *     block-model estimates (the owner of every processor-space coordinate, then
 *     per block boundary the halo cells times the face area where the owners --
 *     or nodes -- on its two sides differ; crossing fractions times the distinct
 *     neighbour offsets otherwise) score them as log2(1 + cells) + lambda *
 *     log2(1 + inter-node cells), and the topk lowest of those are evaluated
 *     exactly.
 * The best of the evaluated candidates is returned.  margin > 0 keeps of the last
 * stage's topk only the candidates scoring at most `margin` above the instance's
 * best score (log2 units: 0.05 = costs within ~3.5 %), so fewer are evaluated;
 * margin = 0 keeps all topk; negative, topk outside 1..4096 or another prefilter:
 * TM_EINVAL.  Everything after the segment upload runs on the device, on `stream`. */
int tm_search(tm_plan* p, tm_ranker* r, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk,
              float lambda, float margin, int64_t* d_best, tm_stencil_cost* d_best_cost, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TASKMAP_H */
