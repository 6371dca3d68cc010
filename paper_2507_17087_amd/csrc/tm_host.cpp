// tm_host.cpp -- host side of libtaskmap: validation, decompose's search,
// descriptor compilation, batch plans and the C entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <functional>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "tm_internal.h"

namespace tmk {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define TM_HIP(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return set_error(TM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ validation

// Forward shape rules of Fig. 6 (split, merge, swap), Sec. 4.2 (decompose) and the
// balance_split reading, from Machine(GPU) = (nodes, gpus).  Records the shape
// before every op (the table-build kernel inverts the ops with them).
int validate_shapes(const tm_candidate* c, Shapes* sh) {
    if (!c) return set_error(TM_EINVAL, "null candidate");
    if (c->lrank < 1 || c->lrank > TM_MAX_LRANK) return set_error(TM_EINVAL, "lrank %d not in 1..4", c->lrank);
    if (c->nodes < 1 || c->gpus_per_node < 1) return set_error(TM_EINVAL, "machine (%d, %d)", c->nodes, c->gpus_per_node);
    if ((int64_t)c->nodes * c->gpus_per_node > TM_MAX_VOLUME)
        return set_error(TM_EOVERFLOW, "more than 2^24 processors");
    if (c->nops < 0 || c->nops > TM_MAX_OPS) return set_error(TM_EINVAL, "nops %d", c->nops);
    int64_t pts = 1;
    for (int d = 0; d < c->lrank; ++d) {
        const int64_t l = c->extent[d];
        if (l < 1 || l > TM_MAX_EXTENT) return set_error(TM_EINVAL, "extent[%d] = %lld", d, (long long)l);
        if (pts > TM_MAX_POINTS / l) return set_error(TM_EOVERFLOW, "more than 2^40 points");
        pts *= l;
    }
    sh->rank[0] = 2;
    sh->size[0][0] = c->nodes;
    sh->size[0][1] = c->gpus_per_node;
    for (int t = 0; t < c->nops; ++t) {
        const tm_op& op = c->ops[t];
        const int r = sh->rank[t];
        const int64_t* s = sh->size[t];
        int64_t* o = sh->size[t + 1];
        int nr = r;
        switch (op.kind) {
            case TM_SPLIT: {
                const int i = op.a;
                const int64_t d = op.b;
                if (i < 0 || i >= r) return set_error(TM_EINVAL, "op %d: split dim %d of rank %d", t, i, r);
                if (d < 1 || s[i] % d) return set_error(TM_EINVAL, "op %d: split factor %lld does not divide %lld", t, (long long)d, (long long)s[i]);
                if (r + 1 > TM_MAX_MRANK) return set_error(TM_EINVAL, "op %d: rank above 8", t);
                nr = r + 1;
                for (int u = 0; u < i; ++u) o[u] = s[u];
                o[i] = d;
                o[i + 1] = s[i] / d;
                for (int u = i + 1; u < r; ++u) o[u + 1] = s[u];
                break;
            }
            case TM_MERGE: {
                const int p = op.a, q = op.b;
                if (p < 0 || p >= q || q >= r) return set_error(TM_EINVAL, "op %d: merge(%d,%d) on rank %d", t, p, q, r);
                nr = r - 1;
                int w = 0;
                for (int u = 0; u < r; ++u)
                    if (u != q) o[w++] = u == p ? s[p] * s[q] : s[u];
                break;
            }
            case TM_SWAP: {
                const int p = op.a, q = op.b;
                if (p < 0 || q < 0 || p >= r || q >= r || p == q)
                    return set_error(TM_EINVAL, "op %d: swap(%d,%d) on rank %d", t, p, q, r);
                for (int u = 0; u < r; ++u) o[u] = s[u];
                std::swap(o[p], o[q]);
                break;
            }
            case TM_BALANCE_SPLIT: {
                const int i = op.a;
                const int64_t d = op.b;
                if (i < 0 || i >= r || d < 1) return set_error(TM_EINVAL, "op %d: balance_split(%d,%lld)", t, i, (long long)d);
                if (d > TM_MAX_VOLUME) return set_error(TM_EOVERFLOW, "op %d: balance_split factor too large", t);
                if (r + 1 > TM_MAX_MRANK) return set_error(TM_EINVAL, "op %d: rank above 8", t);
                nr = r + 1;
                for (int u = 0; u < i; ++u) o[u] = s[u];
                o[i] = d;
                o[i + 1] = (s[i] + d - 1) / d;
                for (int u = i + 1; u < r; ++u) o[u + 1] = s[u];
                break;
            }
            case TM_DECOMPOSE: {
                const int i = op.a, k = op.nf;
                if (i < 0 || i >= r || k < 1 || k > TM_MAX_LRANK)
                    return set_error(TM_EINVAL, "op %d: decompose dim %d with %d factors", t, i, k);
                if (r + k - 1 > TM_MAX_MRANK) return set_error(TM_EINVAL, "op %d: rank above 8", t);
                int64_t prod = 1;
                for (int m = 0; m < k; ++m) {
                    if (op.f[m] < 1) return set_error(TM_EINVAL, "op %d: factor %d", t, op.f[m]);
                    prod *= op.f[m];
                    if (prod > s[i]) return set_error(TM_EINVAL, "op %d: factors exceed %lld", t, (long long)s[i]);
                }
                if (prod != s[i]) return set_error(TM_EINVAL, "op %d: factor product %lld != %lld", t, (long long)prod, (long long)s[i]);
                nr = r + k - 1;
                for (int u = 0; u < i; ++u) o[u] = s[u];
                for (int m = 0; m < k; ++m) o[i + m] = op.f[m];
                for (int u = i + 1; u < r; ++u) o[u + k - 1] = s[u];
                break;
            }
            default:
                return set_error(TM_EINVAL, "op %d: unknown kind %d", t, op.kind);
        }
        sh->rank[t + 1] = nr;
        int64_t vol = 1;
        for (int u = 0; u < nr; ++u) vol *= o[u];
        if (vol > TM_MAX_VOLUME) return set_error(TM_EOVERFLOW, "op %d: processor space volume above 2^24", t);
    }
    const int fr = sh->rank[c->nops];
    if (c->mrank != fr) return set_error(TM_EINVAL, "mrank %d but the final rank is %d", c->mrank, fr);
    for (int j = 0; j < fr; ++j) {
        if (c->proj_src[j] < 0 || c->proj_src[j] >= c->lrank)
            return set_error(TM_EINVAL, "proj_src[%d] = %d", j, (int)c->proj_src[j]);
        if (c->proj_mode[j] != TM_BLOCK && c->proj_mode[j] != TM_CYCLIC)
            return set_error(TM_EINVAL, "proj_mode[%d] = %d", j, (int)c->proj_mode[j]);
    }
    return TM_OK;
}

static int bits_for(int64_t g) {
    int b = 0;
    while ((int64_t(1) << b) < g) ++b;
    return b;
}

int fill_devcand(const tm_candidate* c, const Shapes& sh, DevCand* d) {
    std::memset(d, 0, sizeof(*d));
    d->lrank = c->lrank;
    d->nops = c->nops;
    d->nodes = c->nodes;
    d->gpus = c->gpus_per_node;
    d->gbits = bits_for(c->gpus_per_node);
    const int fr = sh.rank[c->nops];
    d->frank = fr;
    int64_t vol = 1;
    for (int j = fr - 1; j >= 0; --j) {
        d->fshape[j] = (int32_t)sh.size[c->nops][j];
        d->fstride[j] = (int32_t)vol;
        vol *= sh.size[c->nops][j];
    }
    d->vol = (int32_t)vol;
    int64_t words = vol, pts = 1;
    for (int k = 0; k < c->lrank; ++k) {
        d->extent[k] = c->extent[k];
        d->coord_off[k] = (int32_t)std::min<int64_t>(words, INT32_MAX);
        words += c->extent[k];
        pts *= c->extent[k];
    }
    d->words = (int32_t)std::min<int64_t>(words, INT32_MAX);
    d->npoints = pts;
    d->L = (int32_t)c->extent[c->lrank - 1];
    d->rows = pts / c->extent[c->lrank - 1];
    for (int j = 0; j < fr; ++j) {
        d->proj_src[j] = c->proj_src[j];
        d->proj_mode[j] = c->proj_mode[j];
    }
    for (int t = 0; t < c->nops; ++t) {
        d->rank[t] = sh.rank[t];
        for (int u = 0; u < sh.rank[t]; ++u) d->shape[t][u] = (int32_t)sh.size[t][u];
        d->op_kind[t] = c->ops[t].kind;
        d->op_a[t] = c->ops[t].a;
        d->op_b[t] = c->ops[t].b;
        d->op_nf[t] = c->ops[t].nf;
        for (int m = 0; m < TM_MAX_LRANK; ++m) d->op_f[t][m] = c->ops[t].f[m];
        // the op's range [lo, hi] in its input shape and the products around it
        const int64_t* s = sh.size[t];
        const int r = sh.rank[t], pa = c->ops[t].a, pb = c->ops[t].b;
        const int kind = c->ops[t].kind;
        const bool pair = kind == TM_MERGE || kind == TM_SWAP;
        const int lo = pair ? std::min(pa, pb) : pa, hi = pair ? std::max(pa, pb) : pa;
        int64_t after = 1, win = 1, mid = 1;
        for (int u = hi + 1; u < r; ++u) after *= s[u];
        for (int u = lo; u <= hi; ++u) win *= s[u];
        for (int u = lo + 1; u < hi; ++u) mid *= s[u];
        int64_t sc = 1, wout = win;
        if (kind == TM_SPLIT) sc = s[pa] / pb;
        if (kind == TM_BALANCE_SPLIT) {
            sc = (s[pa] + pb - 1) / pb;
            wout = (int64_t)pb * sc;
        }
        d->inv_lo[t] = (int32_t)after;
        d->inv_win[t] = (int32_t)win;
        d->inv_wout[t] = (int32_t)wout;
        d->inv_mid[t] = (int32_t)mid;
        d->inv_c[t] = (int32_t)sc;
    }
    return words > INT32_MAX ? TM_EOVERFLOW : TM_OK;
}

// ------------------------------------------------------------------ decompose's search

static int check_pk(int64_t P, int32_t k) {
    if (P < 1 || P > TM_MAX_VOLUME) return set_error(TM_EINVAL, "P = %lld not in 1..2^24", (long long)P);
    if (k < 1 || k > TM_MAX_LRANK) return set_error(TM_EINVAL, "k = %d not in 1..4", k);
    return TM_OK;
}

// Prime factorization P = prod p_j^{a_j} (trial division), primes ascending.
static void factorize(int64_t P, std::vector<std::pair<int64_t, int>>& pe) {
    pe.clear();
    for (int64_t p = 2; p * p <= P; ++p) {
        int e = 0;
        while (P % p == 0) {
            P /= p;
            ++e;
        }
        if (e) pe.push_back({p, e});
    }
    if (P > 1) pe.push_back({P, 1});
}

// Sec. 4.3: distribute each prime's exponent over the k dims (stars and bars) and
// take the Cartesian product over primes; then sort lexicographically.
static void all_factorizations(int64_t P, int k, std::vector<std::array<int32_t, 4>>& out) {
    std::vector<std::pair<int64_t, int>> pe;
    factorize(P, pe);
    out.assign(1, {1, 1, 1, 1});
    for (auto& [p, a] : pe) {
        // all compositions of a into k non-negative parts
        std::vector<std::array<int, 4>> comps;
        std::array<int, 4> cur{0, 0, 0, 0};
        std::function<void(int, int)> rec = [&](int pos, int left) {
            if (pos == k - 1) {
                cur[pos] = left;
                comps.push_back(cur);
                return;
            }
            for (int x = 0; x <= left; ++x) {
                cur[pos] = x;
                rec(pos + 1, left - x);
            }
        };
        rec(0, a);
        std::vector<std::array<int32_t, 4>> next;
        next.reserve(out.size() * comps.size());
        for (auto& f : out)
            for (auto& cp : comps) {
                std::array<int32_t, 4> g = f;
                for (int m = 0; m < k; ++m)
                    for (int e = 0; e < cp[m]; ++e) g[m] *= (int32_t)p;
                next.push_back(g);
            }
        out.swap(next);
    }
    std::sort(out.begin(), out.end(), [k](const std::array<int32_t, 4>& x, const std::array<int32_t, 4>& y) {
        for (int m = 0; m < k; ++m)
            if (x[m] != y[m]) return x[m] < y[m];
        return false;
    });
}

}  // namespace tmk

using namespace tmk;

extern "C" {

int tm_abi_version(void) { return TM_ABI_VERSION; }
int tm_candidate_size(void) { return (int)sizeof(tm_candidate); }
const char* tm_last_error(void) { return g_err; }

int tm_validate(const tm_candidate* c, int32_t* final_shape, int32_t* final_rank) {
    Shapes sh;
    const int rc = validate_shapes(c, &sh);
    if (rc != TM_OK) return rc;
    const int fr = sh.rank[c->nops];
    if (final_rank) *final_rank = fr;
    if (final_shape)
        for (int j = 0; j < fr; ++j) final_shape[j] = (int32_t)sh.size[c->nops][j];
    return TM_OK;
}

int tm_enumerate_factorizations(int64_t P, int32_t k, int32_t* out, int64_t cap, int64_t* count) {
    int rc = check_pk(P, k);
    if (rc != TM_OK) return rc;
    if (cap < 0 || (cap > 0 && !out)) return set_error(TM_EINVAL, "bad output buffer");
    std::vector<std::array<int32_t, 4>> all;
    all_factorizations(P, k, all);
    if (count) *count = (int64_t)all.size();
    if ((int64_t)all.size() > cap)
        return set_error(TM_ECAPACITY, "%zu factorizations, capacity %lld", all.size(), (long long)cap);
    for (size_t i = 0; i < all.size(); ++i)
        for (int m = 0; m < k; ++m) out[i * k + m] = all[i][m];
    return TM_OK;
}

int tm_decompose_argmin(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo, int32_t* out_f) {
    int rc = check_pk(P, k);
    if (rc != TM_OK) return rc;
    if (!extent || !halo || !out_f) return set_error(TM_EINVAL, "null argument");
    for (int m = 0; m < k; ++m) {
        if (extent[m] < 1 || extent[m] > TM_MAX_EXTENT) return set_error(TM_EINVAL, "extent[%d]", m);
        if (halo[m] < 0 || halo[m] > TM_MAX_HALO) return set_error(TM_EINVAL, "halo[%d]", m);
    }
    std::vector<std::array<int32_t, 4>> all;
    all_factorizations(P, k, all);
    // objective sum_m h_m f_m prod_{j!=m} l_j, exact in 128 bits; enumeration order is
    // lexicographic, so the first minimum is the lexicographically smallest
    __int128 best = 0;
    int64_t bi = -1;
    for (size_t i = 0; i < all.size(); ++i) {
        __int128 v = 0;
        for (int m = 0; m < k; ++m) {
            __int128 term = (__int128)halo[m] * all[i][m];
            for (int j = 0; j < k; ++j)
                if (j != m && __builtin_mul_overflow(term, (__int128)extent[j], &term))
                    return set_error(TM_EOVERFLOW, "objective overflows 128 bits");
            if (__builtin_add_overflow(v, term, &v)) return set_error(TM_EOVERFLOW, "objective overflows 128 bits");
        }
        if (bi < 0 || v < best) {
            best = v;
            bi = (int64_t)i;
        }
    }
    for (int m = 0; m < k; ++m) out_f[m] = all[bi][m];
    return TM_OK;
}

int tm_transpose_target(const tm_candidate* c, int32_t dim, int32_t into, tm_candidate* out) {
    if (!c || !out) return set_error(TM_EINVAL, "null argument");
    int32_t shape[TM_MAX_MRANK], rank = 0;
    int rc = tm_validate(c, shape, &rank);
    if (rc != TM_OK) return rc;
    if (dim < 0 || dim >= c->lrank || into < 0 || into >= c->lrank || dim == into)
        return set_error(TM_EINVAL, "transpose dims %d into %d", dim, into);
    int jn = -1, jt = -1, cn = 0, ct = 0;
    for (int j = 0; j < c->mrank; ++j) {
        if (c->proj_src[j] == dim) { jn = j; ++cn; }
        if (c->proj_src[j] == into) { jt = j; ++ct; }
    }
    if (cn != 1 || ct != 1) return set_error(TM_EINVAL, "each transpose dim must be projected onto one final dim");
    if (c->proj_mode[jn] != TM_BLOCK || c->proj_mode[jt] != TM_BLOCK)
        return set_error(TM_EINVAL, "transpose dims must be block-projected");
    tm_candidate r = *c;
    int8_t src[TM_MAX_MRANK], mode[TM_MAX_MRANK];
    for (int j = 0; j < c->mrank; ++j) {
        src[j] = c->proj_src[j];
        mode[j] = c->proj_mode[j];
    }
    const int add = jn > jt ? 2 : 1;
    if (r.nops + add > TM_MAX_OPS) return set_error(TM_EINVAL, "no room for %d more ops", add);
    auto push = [&](int32_t kind, int32_t a, int32_t b) {
        tm_op& op = r.ops[r.nops++];
        std::memset(&op, 0, sizeof(op));
        op.kind = kind;
        op.a = a;
        op.b = b;
    };
    if (jn > jt) {  // the final dim of `dim` goes first: merge's lower index is its fast part
        push(TM_SWAP, jt, jn);
        std::swap(src[jn], src[jt]);
        std::swap(mode[jn], mode[jt]);
        std::swap(jn, jt);
    }
    push(TM_MERGE, jn, jt);
    src[jn] = (int8_t)into;
    mode[jn] = TM_BLOCK;
    for (int j = jt; j + 1 < c->mrank; ++j) {
        src[j] = src[j + 1];
        mode[j] = mode[j + 1];
    }
    r.mrank = c->mrank - 1;
    for (int j = 0; j < TM_MAX_MRANK; ++j) {
        r.proj_src[j] = j < r.mrank ? src[j] : 0;
        r.proj_mode[j] = j < r.mrank ? mode[j] : 0;
    }
    rc = tm_validate(&r, shape, &rank);
    if (rc != TM_OK) return rc;
    *out = r;
    return TM_OK;
}

int tm_decompose_argmin_transpose(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo,
                                  int32_t transpose_mask, int32_t* out_f) {
    int rc = check_pk(P, k);
    if (rc != TM_OK) return rc;
    if (!extent || !halo || !out_f) return set_error(TM_EINVAL, "null argument");
    if (transpose_mask < 0 || transpose_mask >= (1 << k)) return set_error(TM_EINVAL, "transpose mask %d", transpose_mask);
    for (int m = 0; m < k; ++m) {
        if (extent[m] < 1 || extent[m] > TM_MAX_EXTENT) return set_error(TM_EINVAL, "extent[%d]", m);
        if (halo[m] < 0 || halo[m] > 255) return set_error(TM_EINVAL, "halo[%d] (at most 255 here)", m);
    }
    __int128 vol = 1;
    for (int m = 0; m < k; ++m) vol *= extent[m];
    if (vol > ((__int128)1 << 40)) return set_error(TM_EOVERFLOW, "more than 2^40 points");
    std::vector<std::array<int32_t, 4>> all;
    all_factorizations(P, k, all);
    // objective = A + vol * sum_{n in T} (f_n - 1) / f_n with A = sum_m h_m f_m
    // prod_{j != m} l_j (< 2^74); as the fraction (A * D + vol * N) / D with
    // D = prod_{n in T} f_n <= P <= 2^24 and N = sum_{n in T} (f_n - 1) D / f_n, two
    // candidates compare by cross-multiplying: every product stays below 2^123
    __int128 best_num = 0, best_den = 1;
    int64_t bi = -1;
    for (size_t i = 0; i < all.size(); ++i) {
        __int128 a = 0, d = 1, nsum = 0;
        for (int m = 0; m < k; ++m) {
            __int128 term = (__int128)halo[m] * all[i][m];
            for (int j = 0; j < k; ++j)
                if (j != m) term *= extent[j];
            a += term;
            if ((transpose_mask >> m) & 1) d *= all[i][m];
        }
        for (int m = 0; m < k; ++m)
            if ((transpose_mask >> m) & 1) nsum += (__int128)(all[i][m] - 1) * (d / all[i][m]);
        const __int128 num = a * d + vol * nsum;
        if (bi < 0 || num * best_den < best_num * d) {
            best_num = num;
            best_den = d;
            bi = (int64_t)i;
        }
    }
    for (int m = 0; m < k; ++m) out_f[m] = all[bi][m];
    return TM_OK;
}

int tm_greedy_grid(int64_t P, int32_t k, int32_t* out_f) {
    int rc = check_pk(P, k);
    if (rc != TM_OK) return rc;
    if (!out_f) return set_error(TM_EINVAL, "null argument");
    // App. A.2: every prime of P, smallest first, multiplies a currently smallest
    // factor.  Equal factors are interchangeable, so the factors are kept in
    // descending order: the prime multiplies the last one, which then moves left
    // past the factors it has overtaken; the result needs no final sort.
    std::vector<std::pair<int64_t, int>> pe;
    factorize(P, pe);
    int64_t f[TM_MAX_LRANK] = {1, 1, 1, 1};
    for (const auto& [p, a] : pe)
        for (int e = 0; e < a; ++e) {
            int j = k - 1;
            const int64_t v = f[j] * p;
            while (j > 0 && f[j - 1] < v) {
                f[j] = f[j - 1];
                --j;
            }
            f[j] = v;
        }
    for (int m = 0; m < k; ++m) out_f[m] = (int32_t)f[m];
    return TM_OK;
}

int tm_workload_greedy(int64_t P, int32_t k, const int64_t* extent, int32_t* out_f) {
    int rc = check_pk(P, k);
    if (rc != TM_OK) return rc;
    if (!extent || !out_f) return set_error(TM_EINVAL, "null argument");
    for (int m = 0; m < k; ++m)
        if (extent[m] < 1 || extent[m] > TM_MAX_EXTENT) return set_error(TM_EINVAL, "extent[%d]", m);
    std::vector<std::pair<int64_t, int>> pe;
    factorize(P, pe);
    int64_t f[4] = {1, 1, 1, 1};
    // w_m = l_m / f_m as exact fractions; spread = max w - min w
    auto less = [](__int128 an, __int128 ad, __int128 bn, __int128 bd) { return an * bd < bn * ad; };
    for (auto& [p, a] : pe)
        for (int e = 0; e < a; ++e) {
            int bj = -1;
            __int128 bn = 0, bd = 1;
            for (int j = 0; j < k; ++j) {
                int64_t g[4];
                for (int m = 0; m < k; ++m) g[m] = f[m];
                g[j] *= p;
                int hi = 0, lo = 0;
                for (int m = 1; m < k; ++m) {
                    if (less(extent[hi], g[hi], extent[m], g[m])) hi = m;
                    if (less(extent[m], g[m], extent[lo], g[lo])) lo = m;
                }
                const __int128 dn = (__int128)extent[hi] * g[lo] - (__int128)extent[lo] * g[hi];
                const __int128 dd = (__int128)g[hi] * g[lo];
                if (bj < 0 || less(dn, dd, bn, bd)) {
                    bj = j;
                    bn = dn;
                    bd = dd;
                }
            }
            f[bj] *= p;
        }
    for (int m = 0; m < k; ++m) out_f[m] = (int32_t)f[m];
    return TM_OK;
}

}  // extern "C"
