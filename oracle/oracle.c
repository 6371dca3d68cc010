/*
 * oracle.c -- plain, slow CPU oracle for exact evaluation of index-task mappings.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path never
 * calls it, and it shares no code with the HIP library: every rule below is
 * written out again here, straight from the paper (Mapple, arXiv 2507.17087).
 *
 * What is computed (all exact integer arithmetic, no floating point):
 *   - processor space shapes after each transformation (Sec. 3.3, Fig. 6 shape
 *     rules; decompose Sec. 4.2; balance_split reading below);
 *   - the processor of one launch point: projection of the point onto the final
 *     processor space (the block mapping of Fig. 1 / Fig. 3, the cyclic mapping of
 *     Fig. 4), then the inverse of every transformation, last to first (Fig. 6
 *     formulas, Sec. 5.2 block1D_x example);
 *   - stencil communication volume: per cell, the set of distinct processors that
 *     own a star neighbour and differ from the cell's owner (Sec. 4.1 example,
 *     Fig. 9 volume, App. A.3 halo widths);
 *   - matmul tile fetches: distinct A[i,k], B[k,j], C[i,j] tiles per processor;
 *   - redistribution volume between two mappings (App. A.3 transposes): cells
 *     whose owner, or owner's node, differs;
 *   - decompose's search: enumeration of ordered factorizations by prime exponents
 *     (Sec. 4.3), the objective of Sec. 4.2 / App. A.3 compared exactly, the
 *     greedy grid of Alg. A1 (App. A.2), the workload greedy of Sec. 4.3.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   balance_split(i,d): never defined in the paper.  Reading: new shape
 *     (..., d, c, ...) with c = ceil(s/d); inverse folds the d*c virtual slots
 *     v = a_i + a_{i+1}*d onto the s real ones by b_i = floor(v*s/(d*c)).
 *     Equal to split(i,d) when d divides s.  PARITY UNPINNED by the paper; pinned
 *     only by its own invariants (equals split when d | s, loads differ by <= 1).
 *   decompose(i, F): the splits split(i+n-1, F[n-1]) for n = 1..k-1 (Sec. 4.2),
 *     so the first factor varies fastest in the inverse.
 *   processor id: node * g + gpu where Machine(GPU) has shape (n, g).
 *   ghost volume: distinct (receiving processor, cell) pairs; non-periodic domain.
 *   inter-node: the receiver's node differs from the cell owner's node.
 *
 * Build: gcc -O2 -std=c11 -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- result codes (same numbers as the public interface; written here again) ---- */
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EOVERFLOW (-2)
#define OR_ECAPACITY (-3)
#define OR_ENOMEM (-4)

#define OR_MAX_LRANK 4
#define OR_MAX_MRANK 8
#define OR_MAX_OPS 8
#define OR_MAX_VOLUME (1LL << 24) /* largest processor-space volume at any step */
#define OR_MAX_EXTENT 2147483647LL
#define OR_MAX_POINTS (1LL << 40)
#define OR_MAX_HALO 65535

enum { OP_SPLIT = 1, OP_MERGE = 2, OP_SWAP = 3, OP_BALANCE_SPLIT = 4, OP_DECOMPOSE = 5 };
enum { PROJ_BLOCK = 0, PROJ_CYCLIC = 1 };

/* Candidate record: 328 bytes, the wire format the tests hand to both sides. */
typedef struct {
    int32_t kind, a, b, nf;
    int32_t f[OR_MAX_LRANK];
} or_op;

typedef struct {
    int32_t lrank, nodes, gpus, nops;
    int64_t extent[OR_MAX_LRANK];
    or_op ops[OR_MAX_OPS];
    int32_t mrank, pad0;
    int8_t proj_src[OR_MAX_MRANK];
    int8_t proj_mode[OR_MAX_MRANK];
} or_cand;

typedef struct {
    int32_t lrank, elem_bytes;
    int32_t halo[OR_MAX_LRANK];
} or_stencil;

/* shapes[t] = processor space shape before op t; shapes[nops] = final shape */
typedef struct {
    int32_t rank[OR_MAX_OPS + 1];
    int64_t size[OR_MAX_OPS + 1][OR_MAX_MRANK];
} or_shapes;

int or_sizeof_candidate(void) { return (int)sizeof(or_cand); }

static int64_t volume_of(const int64_t* s, int r) {
    int64_t v = 1;
    for (int t = 0; t < r; t++) v *= s[t];
    return v;
}

/* Shape rules of every transformation, applied forward from Machine(GPU) = (n, g). */
static int compute_shapes(const or_cand* c, or_shapes* sh) {
    if (c->lrank < 1 || c->lrank > OR_MAX_LRANK) return OR_EINVAL;
    if (c->nodes < 1 || c->gpus < 1) return OR_EINVAL;
    if ((int64_t)c->nodes * (int64_t)c->gpus > OR_MAX_VOLUME) return OR_EOVERFLOW;
    if (c->nops < 0 || c->nops > OR_MAX_OPS) return OR_EINVAL;
    int64_t points = 1;
    for (int d = 0; d < c->lrank; d++) {
        if (c->extent[d] < 1 || c->extent[d] > OR_MAX_EXTENT) return OR_EINVAL;
        if (points > OR_MAX_POINTS / c->extent[d]) return OR_EOVERFLOW;
        points *= c->extent[d];
    }
    sh->rank[0] = 2;
    sh->size[0][0] = c->nodes;
    sh->size[0][1] = c->gpus;
    for (int t = 0; t < c->nops; t++) {
        const or_op* op = &c->ops[t];
        int r = sh->rank[t];
        const int64_t* s = sh->size[t];
        int64_t* o = sh->size[t + 1];
        int nr;
        if (op->kind == OP_SPLIT) {
            /* split(i,d): (.., s_i, ..) -> (.., d, s_i/d, ..); d must divide s_i */
            int i = op->a;
            int64_t d = op->b;
            if (i < 0 || i >= r || d < 1) return OR_EINVAL;
            if (s[i] % d != 0) return OR_EINVAL;
            if (r + 1 > OR_MAX_MRANK) return OR_EINVAL;
            nr = r + 1;
            for (int u = 0; u < i; u++) o[u] = s[u];
            o[i] = d;
            o[i + 1] = s[i] / d;
            for (int u = i + 1; u < r; u++) o[u + 1] = s[u];
        } else if (op->kind == OP_MERGE) {
            /* merge(p,q), p < q: dims p and q fused at position p, q removed */
            int p = op->a, q = op->b;
            if (p < 0 || q >= r || p >= q) return OR_EINVAL;
            nr = r - 1;
            int w = 0;
            for (int u = 0; u < r; u++) {
                if (u == q) continue;
                o[w++] = (u == p) ? s[p] * s[q] : s[u];
            }
        } else if (op->kind == OP_SWAP) {
            int p = op->a, q = op->b;
            if (p < 0 || q < 0 || p >= r || q >= r || p == q) return OR_EINVAL;
            nr = r;
            for (int u = 0; u < r; u++) o[u] = s[u];
            o[p] = s[q];
            o[q] = s[p];
        } else if (op->kind == OP_BALANCE_SPLIT) {
            /* balance_split(i,d): (.., s_i, ..) -> (.., d, ceil(s_i/d), ..) */
            int i = op->a;
            int64_t d = op->b;
            if (i < 0 || i >= r || d < 1) return OR_EINVAL;
            if (d > OR_MAX_VOLUME) return OR_EOVERFLOW;
            if (r + 1 > OR_MAX_MRANK) return OR_EINVAL;
            nr = r + 1;
            for (int u = 0; u < i; u++) o[u] = s[u];
            o[i] = d;
            o[i + 1] = (s[i] + d - 1) / d;
            for (int u = i + 1; u < r; u++) o[u + 1] = s[u];
        } else if (op->kind == OP_DECOMPOSE) {
            /* decompose(i,F): s_i replaced by F[0..k), product of F must be s_i */
            int i = op->a, k = op->nf;
            if (i < 0 || i >= r || k < 1 || k > OR_MAX_LRANK) return OR_EINVAL;
            if (r + k - 1 > OR_MAX_MRANK) return OR_EINVAL;
            int64_t prod = 1;
            for (int m = 0; m < k; m++) {
                if (op->f[m] < 1) return OR_EINVAL;
                prod *= op->f[m];
                if (prod > s[i]) return OR_EINVAL;
            }
            if (prod != s[i]) return OR_EINVAL;
            nr = r + k - 1;
            for (int u = 0; u < i; u++) o[u] = s[u];
            for (int m = 0; m < k; m++) o[i + m] = op->f[m];
            for (int u = i + 1; u < r; u++) o[u + k - 1] = s[u];
        } else {
            return OR_EINVAL;
        }
        sh->rank[t + 1] = nr;
        if (volume_of(o, nr) > OR_MAX_VOLUME) return OR_EOVERFLOW;
    }
    int fr = sh->rank[c->nops];
    if (c->mrank != fr) return OR_EINVAL;
    for (int j = 0; j < fr; j++) {
        if (c->proj_src[j] < 0 || c->proj_src[j] >= c->lrank) return OR_EINVAL;
        if (c->proj_mode[j] != PROJ_BLOCK && c->proj_mode[j] != PROJ_CYCLIC) return OR_EINVAL;
    }
    return OR_OK;
}

int or_validate(const or_cand* c, int32_t* final_shape, int32_t* final_rank) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    int fr = sh.rank[c->nops];
    if (final_rank) *final_rank = fr;
    if (final_shape)
        for (int j = 0; j < fr; j++) final_shape[j] = (int32_t)sh.size[c->nops][j];
    return OR_OK;
}

/* Undo transformation t: a is an index of the space after op t, b of the one before. */
static void invert_op(const or_op* op, const int64_t* before, int rank_before,
                      const int64_t* a, int64_t* b) {
    int r = rank_before;
    if (op->kind == OP_SPLIT) {
        /* Fig. 6: b_t = a_t (t<i), a_i + a_{i+1} d (t=i), a_{t+1} (t>i) */
        int i = op->a;
        int64_t d = op->b;
        for (int u = 0; u < i; u++) b[u] = a[u];
        b[i] = a[i] + a[i + 1] * d;
        for (int u = i + 1; u < r; u++) b[u] = a[u + 1];
    } else if (op->kind == OP_MERGE) {
        /* Fig. 6: b_p = a_p mod s_p, b_q = floor(a_p / s_p), others shift back */
        int p = op->a, q = op->b;
        for (int u = 0; u < r; u++) {
            if (u < p || (u > p && u < q)) b[u] = a[u];
            else if (u == p) b[u] = a[p] % before[p];
            else if (u == q) b[u] = a[p] / before[p];
            else b[u] = a[u - 1];
        }
    } else if (op->kind == OP_SWAP) {
        int p = op->a, q = op->b;
        for (int u = 0; u < r; u++) b[u] = a[u];
        b[p] = a[q];
        b[q] = a[p];
    } else if (op->kind == OP_BALANCE_SPLIT) {
        /* reading: v = a_i + a_{i+1} d over d*c virtual slots, folded onto s real ones */
        int i = op->a;
        int64_t d = op->b;
        int64_t s = before[i];
        int64_t cc = (s + d - 1) / d;
        int64_t v = a[i] + a[i + 1] * d;
        for (int u = 0; u < i; u++) b[u] = a[u];
        b[i] = (v * s) / (d * cc);
        for (int u = i + 1; u < r; u++) b[u] = a[u + 1];
    } else { /* OP_DECOMPOSE: the composed splits, first factor fastest */
        int i = op->a, k = op->nf;
        int64_t acc = 0;
        for (int m = k - 1; m >= 0; m--) acc = acc * op->f[m] + a[i + m];
        for (int u = 0; u < i; u++) b[u] = a[u];
        b[i] = acc;
        for (int u = i + 1; u < r; u++) b[u] = a[u + k - 1];
    }
}

/* The processor of one launch point: projection, then the inverse chain. */
static void owner_of_point(const or_cand* c, const or_shapes* sh, const int64_t* ip,
                           int32_t* node, int32_t* gpu) {
    int64_t cur[OR_MAX_MRANK], prev[OR_MAX_MRANK];
    int fr = sh->rank[c->nops];
    const int64_t* fs = sh->size[c->nops];
    for (int j = 0; j < fr; j++) {
        int64_t x = ip[(int)c->proj_src[j]];
        int64_t l = c->extent[(int)c->proj_src[j]];
        if (c->proj_mode[j] == PROJ_BLOCK) cur[j] = (x * fs[j]) / l; /* point * m.size / space */
        else cur[j] = x % fs[j];                                       /* round robin */
    }
    for (int t = c->nops - 1; t >= 0; t--) {
        invert_op(&c->ops[t], sh->size[t], sh->rank[t], cur, prev);
        for (int u = 0; u < sh->rank[t]; u++) cur[u] = prev[u];
    }
    *node = (int32_t)cur[0];
    *gpu = (int32_t)cur[1];
}

int or_point_owner(const or_cand* c, const int64_t* ip, int32_t* node, int32_t* gpu) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    for (int d = 0; d < c->lrank; d++)
        if (ip[d] < 0 || ip[d] >= c->extent[d]) return OR_EINVAL;
    owner_of_point(c, &sh, ip, node, gpu);
    return OR_OK;
}

static int64_t n_points(const or_cand* c) {
    int64_t n = 1;
    for (int d = 0; d < c->lrank; d++) n *= c->extent[d];
    return n;
}

static void unflatten(const or_cand* c, int64_t flat, int64_t* ip) {
    for (int d = c->lrank - 1; d >= 0; d--) {
        ip[d] = flat % c->extent[d];
        flat /= c->extent[d];
    }
}

/* Processor id (node*g + gpu) of every launch point, C order (last dim fastest). */
int or_proc_map(const or_cand* c, int32_t* out, int64_t len) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    int64_t np = n_points(c);
    if (len != np) return OR_ECAPACITY;
    int64_t ip[OR_MAX_LRANK];
    for (int64_t f = 0; f < np; f++) {
        int32_t node, gpu;
        unflatten(c, f, ip);
        owner_of_point(c, &sh, ip, &node, &gpu);
        out[f] = node * c->gpus + gpu;
    }
    return OR_OK;
}

/* Processor id for every coordinate of the final processor space, C order. */
int or_chain_table(const or_cand* c, int32_t* out, int64_t cap, int64_t* count) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    int fr = sh.rank[c->nops];
    const int64_t* fs = sh.size[c->nops];
    int64_t vol = volume_of(fs, fr);
    if (count) *count = vol;
    if (cap < vol) return OR_ECAPACITY;
    int64_t cur[OR_MAX_MRANK], prev[OR_MAX_MRANK];
    for (int64_t v = 0; v < vol; v++) {
        int64_t rem = v;
        for (int j = fr - 1; j >= 0; j--) {
            cur[j] = rem % fs[j];
            rem /= fs[j];
        }
        for (int t = c->nops - 1; t >= 0; t--) {
            invert_op(&c->ops[t], sh.size[t], sh.rank[t], cur, prev);
            for (int u = 0; u < sh.rank[t]; u++) cur[u] = prev[u];
        }
        out[v] = (int32_t)(cur[0] * c->gpus + cur[1]);
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Stencil ghost volume.  For every cell q: G(q) = distinct owners of the
 * in-domain star neighbours q +- s e_m (1 <= s <= h_m), minus owner(q).
 * ghost += |G(q)|; inter += |{P in G(q) : node(P) != node(owner(q))}|.
 * --------------------------------------------------------------------------- */
#define OR_MATERIALISE_LIMIT (1LL << 28)

int or_stencil_cost(const or_cand* c, const or_stencil* st, int64_t* out4) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    if (st->lrank != c->lrank || st->elem_bytes < 0) return OR_EINVAL;
    int nh = 0;
    for (int d = 0; d < c->lrank; d++) {
        if (st->halo[d] < 0 || st->halo[d] > OR_MAX_HALO) return OR_EINVAL;
        nh += 2 * st->halo[d];
    }
    int64_t np = n_points(c);
    int32_t* own = NULL;
    if (np <= OR_MATERIALISE_LIMIT) {
        own = (int32_t*)malloc((size_t)np * sizeof(int32_t));
        if (!own) return OR_ENOMEM;
        rc = or_proc_map(c, own, np);
        if (rc != OR_OK) { free(own); return rc; }
    }
    int32_t* seen = (int32_t*)malloc((size_t)(nh > 0 ? nh : 1) * sizeof(int32_t));
    if (!seen) { free(own); return OR_ENOMEM; }
    int64_t ghost = 0, inter = 0;
    int64_t ip[OR_MAX_LRANK], jp[OR_MAX_LRANK];
    int g = c->gpus;
    for (int64_t f = 0; f < np; f++) {
        unflatten(c, f, ip);
        int32_t oq;
        if (own) oq = own[f];
        else { int32_t nd, gp; owner_of_point(c, &sh, ip, &nd, &gp); oq = nd * g + gp; }
        int ns = 0;
        for (int m = 0; m < c->lrank; m++) {
            for (int s = 1; s <= st->halo[m]; s++) {
                for (int dir = -1; dir <= 1; dir += 2) {
                    int64_t x = ip[m] + dir * (int64_t)s;
                    if (x < 0 || x >= c->extent[m]) continue; /* non-periodic */
                    for (int d = 0; d < c->lrank; d++) jp[d] = ip[d];
                    jp[m] = x;
                    int32_t op_;
                    if (own) {
                        int64_t jf = 0;
                        for (int d = 0; d < c->lrank; d++) jf = jf * c->extent[d] + jp[d];
                        op_ = own[jf];
                    } else {
                        int32_t nd, gp;
                        owner_of_point(c, &sh, jp, &nd, &gp);
                        op_ = nd * g + gp;
                    }
                    if (op_ == oq) continue;
                    int dup = 0;
                    for (int u = 0; u < ns; u++) if (seen[u] == op_) dup = 1;
                    if (!dup) seen[ns++] = op_;
                }
            }
        }
        ghost += ns;
        for (int u = 0; u < ns; u++)
            if (seen[u] / g != oq / g) inter++;
    }
    free(seen);
    free(own);
    out4[0] = ghost;
    out4[1] = inter;
    out4[2] = ghost * st->elem_bytes;
    out4[3] = inter * st->elem_bytes;
    return OR_OK;
}

/* Node-level exchange volume (the per-node de-duplicated inter-node count used
 * with two-level mappings, where a node receives each remote cell once however many
 * of its GPUs read it): for every cell, the distinct nodes, other than the node
 * owning the cell, that own one of its star neighbours (halo[m] cells along each
 * axis, non-periodic).  out4 = {cells, cells, bytes, bytes}: every such transfer
 * crosses nodes. */
int or_stencil_node_cost(const or_cand* c, const or_stencil* st, int64_t* out4) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    if (st->lrank != c->lrank || st->elem_bytes < 0) return OR_EINVAL;
    int nh = 0;
    for (int d = 0; d < c->lrank; d++) {
        if (st->halo[d] < 0 || st->halo[d] > OR_MAX_HALO) return OR_EINVAL;
        nh += 2 * st->halo[d];
    }
    int64_t np = n_points(c);
    int32_t* own = NULL;
    if (np <= OR_MATERIALISE_LIMIT) {
        own = (int32_t*)malloc((size_t)np * sizeof(int32_t));
        if (!own) return OR_ENOMEM;
        rc = or_proc_map(c, own, np);
        if (rc != OR_OK) { free(own); return rc; }
    }
    int32_t* seen = (int32_t*)malloc((size_t)(nh > 0 ? nh : 1) * sizeof(int32_t));
    if (!seen) { free(own); return OR_ENOMEM; }
    int64_t cells = 0;
    int64_t ip[OR_MAX_LRANK], jp[OR_MAX_LRANK];
    int g = c->gpus;
    for (int64_t f = 0; f < np; f++) {
        unflatten(c, f, ip);
        int32_t node_q;
        if (own) node_q = own[f] / g;
        else { int32_t nd, gp; owner_of_point(c, &sh, ip, &nd, &gp); node_q = nd; }
        int ns = 0;
        for (int m = 0; m < c->lrank; m++) {
            for (int s = 1; s <= st->halo[m]; s++) {
                for (int dir = -1; dir <= 1; dir += 2) {
                    int64_t x = ip[m] + dir * (int64_t)s;
                    if (x < 0 || x >= c->extent[m]) continue;
                    for (int d = 0; d < c->lrank; d++) jp[d] = ip[d];
                    jp[m] = x;
                    int32_t node_p;
                    if (own) {
                        int64_t jf = 0;
                        for (int d = 0; d < c->lrank; d++) jf = jf * c->extent[d] + jp[d];
                        node_p = own[jf] / g;
                    } else {
                        int32_t nd, gp;
                        owner_of_point(c, &sh, jp, &nd, &gp);
                        node_p = nd;
                    }
                    if (node_p == node_q) continue;
                    int dup = 0;
                    for (int u = 0; u < ns; u++) if (seen[u] == node_p) dup = 1;
                    if (!dup) seen[ns++] = node_p;
                }
            }
        }
        cells += ns;
    }
    free(seen);
    free(own);
    out4[0] = cells;
    out4[1] = cells;
    out4[2] = cells * st->elem_bytes;
    out4[3] = cells * st->elem_bytes;
    return OR_OK;
}

int or_stencil_node_cost_batch(const or_cand* c, int64_t n, const or_stencil* st, int64_t* out4n) {
    for (int64_t i = 0; i < n; i++) {
        int rc = or_stencil_node_cost(&c[i], st, out4n + 4 * i);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* Stencil cost of a batch, one candidate after the other. */
int or_stencil_cost_batch(const or_cand* c, int64_t n, const or_stencil* st, int64_t* out4n) {
    for (int64_t i = 0; i < n; i++) {
        int rc = or_stencil_cost(&c[i], st, out4n + 4 * i);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Redistribution volume between two mappings a and b of the same launch domain on
 * the same machine: every cell's data moves from its owner under a to its owner
 * under b.  A transpose by all-to-all exchanges along one dimension (App. A.3) is
 * such a redistribution, from a mapping to its pencil-transposed image (built by
 * the caller).  moved = cells whose two owners differ; inter = cells whose two
 * owners sit on different nodes.  out4 = {moved, inter, moved * elem_bytes,
 * inter * elem_bytes}.
 * --------------------------------------------------------------------------- */
int or_redistribution_cost(const or_cand* a, const or_cand* b, int64_t elem_bytes, int64_t* out4) {
    or_shapes sa, sb;
    int rc = compute_shapes(a, &sa);
    if (rc != OR_OK) return rc;
    rc = compute_shapes(b, &sb);
    if (rc != OR_OK) return rc;
    if (elem_bytes < 0 || a->lrank != b->lrank || a->nodes != b->nodes || a->gpus != b->gpus) return OR_EINVAL;
    for (int d = 0; d < a->lrank; d++)
        if (a->extent[d] != b->extent[d]) return OR_EINVAL;
    int64_t np = n_points(a), moved = 0, inter = 0;
    int64_t ip[OR_MAX_LRANK];
    for (int64_t f = 0; f < np; f++) {
        int32_t na, ga, nb, gb;
        unflatten(a, f, ip);
        owner_of_point(a, &sa, ip, &na, &ga);
        owner_of_point(b, &sb, ip, &nb, &gb);
        if (na != nb || ga != gb) moved++;
        if (na != nb) inter++;
    }
    out4[0] = moved;
    out4[1] = inter;
    out4[2] = moved * elem_bytes;
    out4[3] = inter * elem_bytes;
    return OR_OK;
}

int or_redistribution_cost_batch(const or_cand* a, const or_cand* b, int64_t n, int64_t elem_bytes,
                                 int64_t* out4n) {
    for (int64_t i = 0; i < n; i++) {
        int rc = or_redistribution_cost(&a[i], &b[i], elem_bytes, out4n + 4 * i);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Matmul tile fetches.  Task (i,j,k) -> processor P touches A[i,k], B[k,j], C[i,j].
 * Per processor: number of distinct tiles of each matrix.
 * out7 = {tilesA, tilesB, tilesC, maxA, maxB, maxC, bytes}; per_proc[P][3].
 * --------------------------------------------------------------------------- */
int or_matmul_cost(const or_cand* c, int64_t tile_bytes, int64_t* per_proc, int64_t* out7) {
    or_shapes sh;
    int rc = compute_shapes(c, &sh);
    if (rc != OR_OK) return rc;
    if (c->lrank != 3 || tile_bytes < 0) return OR_EINVAL;
    int64_t Ti = c->extent[0], Tj = c->extent[1], Tk = c->extent[2];
    int64_t P = (int64_t)c->nodes * c->gpus;
    int64_t nA = Ti * Tk, nB = Tk * Tj, nC = Ti * Tj;
    /* one bit per (processor, tile) for each matrix */
    int64_t wA = (nA + 63) / 64, wB = (nB + 63) / 64, wC = (nC + 63) / 64;
    uint64_t* bA = (uint64_t*)calloc((size_t)(P * wA), 8);
    uint64_t* bB = (uint64_t*)calloc((size_t)(P * wB), 8);
    uint64_t* bC = (uint64_t*)calloc((size_t)(P * wC), 8);
    if (!bA || !bB || !bC) { free(bA); free(bB); free(bC); return OR_ENOMEM; }
    int64_t ip[3];
    for (ip[0] = 0; ip[0] < Ti; ip[0]++)
        for (ip[1] = 0; ip[1] < Tj; ip[1]++)
            for (ip[2] = 0; ip[2] < Tk; ip[2]++) {
                int32_t nd, gp;
                owner_of_point(c, &sh, ip, &nd, &gp);
                int64_t p = (int64_t)nd * c->gpus + gp;
                int64_t ta = ip[0] * Tk + ip[2]; /* A[i,k] */
                int64_t tb = ip[2] * Tj + ip[1]; /* B[k,j] */
                int64_t tc = ip[0] * Tj + ip[1]; /* C[i,j] */
                bA[p * wA + ta / 64] |= 1ULL << (ta % 64);
                bB[p * wB + tb / 64] |= 1ULL << (tb % 64);
                bC[p * wC + tc / 64] |= 1ULL << (tc % 64);
            }
    int64_t tot[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    for (int64_t p = 0; p < P; p++) {
        int64_t cnt[3] = {0, 0, 0};
        for (int64_t w = 0; w < wA; w++) cnt[0] += __builtin_popcountll(bA[p * wA + w]);
        for (int64_t w = 0; w < wB; w++) cnt[1] += __builtin_popcountll(bB[p * wB + w]);
        for (int64_t w = 0; w < wC; w++) cnt[2] += __builtin_popcountll(bC[p * wC + w]);
        for (int m = 0; m < 3; m++) {
            if (per_proc) per_proc[p * 3 + m] = cnt[m];
            tot[m] += cnt[m];
            if (cnt[m] > mx[m]) mx[m] = cnt[m];
        }
    }
    free(bA); free(bB); free(bC);
    for (int m = 0; m < 3; m++) { out7[m] = tot[m]; out7[3 + m] = mx[m]; }
    out7[6] = (tot[0] + tot[1] + tot[2]) * tile_bytes;
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * decompose's search space (Sec. 4.3): all ordered k-tuples with product P.
 * A plain recursive walk over divisors, smallest first, gives lexicographic
 * ascending order.
 * --------------------------------------------------------------------------- */
static void enum_rec(int64_t rem, int k, int pos, int32_t* cur, int32_t* out, int64_t cap,
                     int64_t* n) {
    if (pos == k - 1) {
        cur[pos] = (int32_t)rem;
        if (*n < cap) memcpy(out + (*n) * k, cur, (size_t)k * sizeof(int32_t));
        (*n)++;
        return;
    }
    for (int64_t d = 1; d <= rem; d++) {
        if (rem % d) continue;
        cur[pos] = (int32_t)d;
        enum_rec(rem / d, k, pos + 1, cur, out, cap, n);
    }
}

int or_enum_factorizations(int64_t P, int32_t k, int32_t* out, int64_t cap, int64_t* count) {
    if (P < 1 || P > OR_MAX_VOLUME || k < 1 || k > OR_MAX_LRANK || cap < 0) return OR_EINVAL;
    int32_t cur[OR_MAX_LRANK];
    int64_t n = 0;
    enum_rec(P, k, 0, cur, out, cap, &n);
    if (count) *count = n;
    return n > cap ? OR_ECAPACITY : OR_OK;
}

/* decompose's objective with halo widths (Sec. 4.2, App. A.3):
 *   V(F) = sum_m h_m * f_m * prod_{j != m} l_j      (exact, 128-bit)
 * argmin over the full enumeration; ties -> lexicographically smallest F. */
static int objective(int k, const int32_t* f, const int64_t* l, const int32_t* h, __int128* val) {
    __int128 v = 0;
    for (int m = 0; m < k; m++) {
        __int128 term = (__int128)h[m] * f[m];
        for (int j = 0; j < k; j++) {
            if (j == m) continue;
            if (__builtin_mul_overflow(term, (__int128)l[j], &term)) return OR_EOVERFLOW;
        }
        if (__builtin_add_overflow(v, term, &v)) return OR_EOVERFLOW;
    }
    *val = v;
    return OR_OK;
}

int or_decompose_argmin(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo,
                        int32_t* out_f) {
    if (P < 1 || P > OR_MAX_VOLUME || k < 1 || k > OR_MAX_LRANK) return OR_EINVAL;
    for (int m = 0; m < k; m++) {
        if (extent[m] < 1 || extent[m] > OR_MAX_EXTENT) return OR_EINVAL;
        if (halo[m] < 0 || halo[m] > OR_MAX_HALO) return OR_EINVAL;
    }
    int64_t n = 0;
    or_enum_factorizations(P, k, NULL, 0, &n);
    int32_t* all = (int32_t*)malloc((size_t)(n * k) * sizeof(int32_t));
    if (!all) return OR_ENOMEM;
    or_enum_factorizations(P, k, all, n, &n);
    int64_t best = -1;
    __int128 bestv = 0;
    for (int64_t i = 0; i < n; i++) {
        __int128 v;
        int rc = objective(k, all + i * k, extent, halo, &v);
        if (rc != OR_OK) { free(all); return rc; }
        if (best < 0 || v < bestv) { best = i; bestv = v; } /* strict: first (lex smallest) wins ties */
    }
    memcpy(out_f, all + best * k, (size_t)k * sizeof(int32_t));
    free(all);
    return OR_OK;
}

/* Ascending list of prime factors with multiplicity (trial division). */
static int prime_factors(int64_t P, int64_t* pr) {
    int n = 0;
    for (int64_t p = 2; p * p <= P; p++)
        while (P % p == 0) { pr[n++] = p; P /= p; }
    if (P > 1) pr[n++] = P;
    return n;
}

/* Alg. A1 (App. A.2): each prime, smallest first, multiplies the currently smallest
 * factor (lowest index on ties); the result is sorted descending. */
int or_greedy_grid(int64_t P, int32_t k, int32_t* out_f) {
    if (P < 1 || P > OR_MAX_VOLUME || k < 1 || k > OR_MAX_LRANK) return OR_EINVAL;
    int64_t pr[64];
    int np = prime_factors(P, pr);
    int64_t f[OR_MAX_LRANK];
    for (int m = 0; m < k; m++) f[m] = 1;
    for (int t = 0; t < np; t++) {
        int j = 0;
        for (int m = 1; m < k; m++) if (f[m] < f[j]) j = m;
        f[j] *= pr[t];
    }
    for (int a = 0; a < k; a++) /* selection sort, descending */
        for (int b = a + 1; b < k; b++)
            if (f[b] > f[a]) { int64_t tmp = f[a]; f[a] = f[b]; f[b] = tmp; }
    for (int m = 0; m < k; m++) out_f[m] = (int32_t)f[m];
    return OR_OK;
}

/* The workload greedy of Sec. 4.3: primes smallest first; each goes to the dimension
 * whose choice minimises max(w) - min(w), w_m = l_m / f_m (exact rationals, lowest
 * index on ties). */
static int frac_less(__int128 an, __int128 ad, __int128 bn, __int128 bd) { return an * bd < bn * ad; }

int or_workload_greedy(int64_t P, int32_t k, const int64_t* extent, int32_t* out_f) {
    if (P < 1 || P > OR_MAX_VOLUME || k < 1 || k > OR_MAX_LRANK) return OR_EINVAL;
    for (int m = 0; m < k; m++)
        if (extent[m] < 1 || extent[m] > OR_MAX_EXTENT) return OR_EINVAL;
    int64_t pr[64];
    int np = prime_factors(P, pr);
    int64_t f[OR_MAX_LRANK];
    for (int m = 0; m < k; m++) f[m] = 1;
    for (int t = 0; t < np; t++) {
        int bestj = -1;
        __int128 bn = 0, bd = 1;
        for (int j = 0; j < k; j++) {
            int64_t g[OR_MAX_LRANK];
            for (int m = 0; m < k; m++) g[m] = f[m];
            g[j] *= pr[t];
            /* spread = max_m l_m/g_m - min_m l_m/g_m */
            int imax = 0, imin = 0;
            for (int m = 1; m < k; m++) {
                if (frac_less(extent[imax], g[imax], extent[m], g[m])) imax = m;
                if (frac_less(extent[m], g[m], extent[imin], g[imin])) imin = m;
            }
            __int128 dn = (__int128)extent[imax] * g[imin] - (__int128)extent[imin] * g[imax];
            __int128 dd = (__int128)g[imax] * g[imin];
            if (bestj < 0 || frac_less(dn, dd, bn, bd)) { bestj = j; bn = dn; bd = dd; }
        }
        f[bestj] *= pr[t];
    }
    for (int m = 0; m < k; m++) out_f[m] = (int32_t)f[m];
    return OR_OK;
}

/* Exhaustive selection: minimum of (bytes, inter_bytes, index). */
int or_select_best(const int64_t* cost4, int64_t n, int64_t* best) {
    if (n < 1) return OR_EINVAL;
    int64_t b = 0;
    for (int64_t i = 1; i < n; i++) {
        const int64_t* x = cost4 + 4 * i;
        const int64_t* y = cost4 + 4 * b;
        if (x[2] < y[2] || (x[2] == y[2] && x[3] < y[3])) b = i;
    }
    *best = b;
    return OR_OK;
}
