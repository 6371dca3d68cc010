/*
 * gen.c -- seeded synthetic candidate generator (inputs only).
 *
 * Draws random candidate mappings: a launch domain, a machine (nodes x GPUs per
 * node), a factorization of the processor count and a short random chain of
 * processor-space transformations.  It evaluates nothing: it computes no
 * processor ids and no communication.  To draw only valid transformation
 * arguments it keeps the forward shape of the processor space as it goes
 * (the shape rules of split / merge / swap / balance_split / decompose), which is
 * the input grammar, not the evaluation.
 *
 * Random numbers: splitmix64 (Steele, Lea & Flood, OOPSLA 2014) and bounded draws
 * by Lemire's multiply-shift with rejection (Lemire, ACM TOMACS 2019, "Fast random
 * integer generation in an interval").  Candidate i uses its own stream derived
 * from (seed, i), so any subset of a batch can be regenerated on its own.
 *
 * Record layout (328 bytes) is the candidate wire format also read by the tests.
 */
#include <stdint.h>
#include <string.h>

typedef struct {
    int32_t kind, a, b, nf;
    int32_t f[4];
} g_op;

typedef struct {
    int32_t lrank, nodes, gpus, nops;
    int64_t extent[4];
    g_op ops[8];
    int32_t mrank, pad0;
    int8_t proj_src[8];
    int8_t proj_mode[8];
} g_cand;

enum { K_SPLIT = 1, K_MERGE = 2, K_SWAP = 3, K_BALANCE = 4, K_DECOMPOSE = 5 };
#define G_MAX_RANK 8
#define G_MAX_VOLUME (1LL << 24)

int gen_sizeof_candidate(void) { return (int)sizeof(g_cand); }

typedef struct { uint64_t s; } rng_t;

static uint64_t sm64(rng_t* r) {
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform integer in [0, n), n >= 1 */
static uint64_t below(rng_t* r, uint64_t n) {
    uint64_t x = sm64(r);
    __uint128_t m = (__uint128_t)x * n;
    uint64_t lo = (uint64_t)m;
    if (lo < n) {
        uint64_t t = (0 - n) % n;
        while (lo < t) {
            x = sm64(r);
            m = (__uint128_t)x * n;
            lo = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}

static void stream_for(rng_t* r, uint64_t seed, uint64_t index) {
    rng_t t = {seed};
    uint64_t a = sm64(&t);
    r->s = a ^ (index * 0xD1B54A32D192ED03ULL);
    (void)sm64(r);
}

/* uniform divisor of v (trial listing) */
static int64_t uniform_divisor(rng_t* r, int64_t v) {
    int64_t divs[4096];
    int n = 0;
    for (int64_t d = 1; d <= v && n < 4096; d++)
        if (v % d == 0) divs[n++] = d;
    return divs[below(r, (uint64_t)n)];
}

/* ordered k-factorizations of P, written as k-tuples to out (up to cap of them);
 * returns how many there are (a divisor walk: the first factor, then the
 * factorizations of what is left) */
static int64_t factorizations(int64_t P, int k, int32_t* prefix, int depth, int32_t* out, int64_t n,
                              int64_t cap) {
    if (depth == k - 1) {
        if (n < cap) {
            for (int m = 0; m < k - 1; m++) out[n * k + m] = prefix[m];
            out[n * k + k - 1] = (int32_t)P;
        }
        return n + 1;
    }
    for (int64_t d = 1; d <= P; d++) {
        if (P % d) continue;
        prefix[depth] = (int32_t)d;
        n = factorizations(P / d, k, prefix, depth + 1, out, n, cap);
    }
    return n;
}

/* random ordered k-factorization of P, uniform over all of them */
static void random_factorization(rng_t* r, int64_t P, int k, int32_t* f) {
    static _Thread_local int32_t all[4 * 8192];
    int32_t prefix[4];
    const int64_t n = factorizations(P, k, prefix, 0, all, 0, 8192);
    const int64_t pick = (int64_t)below(r, (uint64_t)(n < 8192 ? n : 8192));
    for (int m = 0; m < k; m++) f[m] = all[pick * k + m];
}

static int64_t vol(const int64_t* s, int r) {
    int64_t v = 1;
    for (int t = 0; t < r; t++) v *= s[t];
    return v;
}

/* draws one random transformation valid for shape s (rank *r); updates the shape.
 * returns 0 if the drawn kind has no valid arguments at this shape. */
static int random_op(rng_t* rg, int64_t* s, int* r, g_op* op) {
    int kind = 1 + (int)below(rg, 4); /* split, merge, swap, balance_split */
    int rank = *r;
    memset(op, 0, sizeof(*op));
    op->kind = kind == 4 ? K_BALANCE : kind;
    if (kind == K_SWAP) {
        if (rank < 2) return 0;
        int p = (int)below(rg, (uint64_t)rank);
        int q = (int)below(rg, (uint64_t)(rank - 1));
        if (q >= p) q++;
        op->a = p;
        op->b = q;
        int64_t t = s[p]; s[p] = s[q]; s[q] = t;
        return 1;
    }
    if (kind == K_MERGE) {
        if (rank < 2) return 0;
        int p = (int)below(rg, (uint64_t)rank);
        int q = (int)below(rg, (uint64_t)(rank - 1));
        if (q >= p) q++;
        if (p > q) { int t = p; p = q; q = t; }
        op->a = p;
        op->b = q;
        int64_t ns[G_MAX_RANK];
        int w = 0;
        for (int u = 0; u < rank; u++) {
            if (u == q) continue;
            ns[w++] = (u == p) ? s[p] * s[q] : s[u];
        }
        memcpy(s, ns, sizeof(int64_t) * (size_t)w);
        *r = rank - 1;
        return 1;
    }
    if (rank + 1 > G_MAX_RANK) return 0;
    int i = (int)below(rg, (uint64_t)rank);
    int64_t d, c;
    if (kind == K_SPLIT) {
        d = uniform_divisor(rg, s[i]);
        c = s[i] / d;
    } else {
        d = 1 + (int64_t)below(rg, (uint64_t)s[i]);
        c = (s[i] + d - 1) / d;
    }
    int64_t ns[G_MAX_RANK];
    for (int u = 0; u < i; u++) ns[u] = s[u];
    ns[i] = d;
    ns[i + 1] = c;
    for (int u = i + 1; u < rank; u++) ns[u + 1] = s[u];
    if (vol(ns, rank + 1) > G_MAX_VOLUME) return 0;
    op->a = i;
    op->b = (int32_t)d;
    memcpy(s, ns, sizeof(int64_t) * (size_t)(rank + 1));
    *r = rank + 1;
    return 1;
}

/* The chain part of a random candidate whose launch rank, domain and machine are
 * set: merge(0,1) + decompose(0, F) with F uniform over the factorizations of
 * nodes * gpus, then 0..max_ops random transformations (redrawn until the final
 * rank is k), then per final dim a cyclic projection with probability cyclic_pct. */
static void draw_chain(rng_t* rg, g_cand* c, int k, int32_t max_ops, int32_t cyclic_pct) {
    int64_t P = (int64_t)c->nodes * c->gpus;
    int32_t f[4];
    random_factorization(rg, P, k, f);
    c->ops[0].kind = K_MERGE; c->ops[0].a = 0; c->ops[0].b = 1;
    c->ops[1].kind = K_DECOMPOSE; c->ops[1].a = 0; c->ops[1].nf = k;
    for (int m = 0; m < k; m++) c->ops[1].f[m] = f[m];
    int ntries = 0;
    for (;;) {
        int64_t s[G_MAX_RANK];
        int r = k;
        for (int m = 0; m < k; m++) s[m] = f[m];
        int nx = (int)below(rg, (uint64_t)(max_ops + 1));
        int ok = 1;
        for (int t = 0; t < nx && ok; t++) ok = random_op(rg, s, &r, &c->ops[2 + t]);
        if (ok && r == k) { c->nops = 2 + nx; break; }
        if (++ntries > 1000) { c->nops = 2; break; } /* fall back to the plain decompose */
    }
    for (int t = c->nops; t < 8; t++) memset(&c->ops[t], 0, sizeof(g_op));
    c->mrank = k;
    for (int j = 0; j < k; j++) {
        c->proj_src[j] = (int8_t)j;
        c->proj_mode[j] = (cyclic_pct > 0 && (int)below(rg, 100) < cyclic_pct) ? 1 : 0;
    }
}

/*
 * Batched random candidates.
 *   k_mask    : bit k set -> launch rank k allowed (e.g. 0b1100 = ranks 2 and 3)
 *   oct_lo/hi : per-dim extent l drawn as octave b uniform in [oct_lo, oct_hi], then
 *               l uniform in [2^b, 2^(b+1))
 *   nodes_max : nodes uniform in [1, nodes_max]
 *   gpus_mask : allowed GPUs per node as a bit set over {1,2,4,8,...} (bit t -> 2^t)
 *   max_ops   : number of random transformations uniform in [0, max_ops]
 *   cyclic_pct: percent chance for each final dim to use the cyclic projection
 */
int gen_random_candidates(uint64_t seed, int64_t first, int64_t n, int32_t k_mask, int32_t oct_lo,
                          int32_t oct_hi, int32_t nodes_max, int32_t gpus_mask, int32_t max_ops,
                          int32_t cyclic_pct, g_cand* out) {
    int ks[8], nk = 0, gs[8], ng = 0;
    for (int k = 1; k <= 4; k++) if (k_mask & (1 << k)) ks[nk++] = k;
    for (int t = 0; t < 8; t++) if (gpus_mask & (1 << t)) gs[ng++] = 1 << t;
    if (nk == 0 || ng == 0 || oct_lo < 0 || oct_hi < oct_lo || oct_hi > 30 || nodes_max < 1 ||
        max_ops < 0 || max_ops > 6)
        return -1;
    for (int64_t idx = 0; idx < n; idx++) {
        rng_t rg;
        stream_for(&rg, seed, (uint64_t)(first + idx));
        g_cand* c = &out[idx];
        memset(c, 0, sizeof(*c));
        int k = ks[below(&rg, (uint64_t)nk)];
        c->lrank = k;
        for (int d = 0; d < k; d++) {
            int b = oct_lo + (int)below(&rg, (uint64_t)(oct_hi - oct_lo + 1));
            int64_t lo = 1LL << b;
            c->extent[d] = lo + (int64_t)below(&rg, (uint64_t)lo);
        }
        c->nodes = 1 + (int32_t)below(&rg, (uint64_t)nodes_max);
        c->gpus = gs[below(&rg, (uint64_t)ng)];
        draw_chain(&rg, c, k, max_ops, cyclic_pct);
    }
    return 0;
}

/*
 * Random chains on one launch domain and machine (a search instance): candidate idx
 * (its own stream, as above) draws only its chain and projections.
 */
int gen_random_chains(uint64_t seed, int64_t first, int64_t n, int32_t k, const int64_t* extent, int32_t nodes,
                      int32_t gpus, int32_t max_ops, int32_t cyclic_pct, g_cand* out) {
    if (k < 1 || k > 4 || nodes < 1 || gpus < 1 || max_ops < 0 || max_ops > 6) return -1;
    for (int64_t idx = 0; idx < n; idx++) {
        rng_t rg;
        stream_for(&rg, seed, (uint64_t)(first + idx));
        g_cand* c = &out[idx];
        memset(c, 0, sizeof(*c));
        c->lrank = k;
        for (int d = 0; d < k; d++) c->extent[d] = extent[d];
        c->nodes = nodes;
        c->gpus = gpus;
        draw_chain(&rg, c, k, max_ops, cyclic_pct);
    }
    return 0;
}
