// fuzz_host.cpp -- seeded differential fuzzing of the library's host layer against
// the oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer (TEST
// INFRASTRUCTURE: built and run by tests/test_sanitize_cpu.py, never part of the
// product).
//
// Cases (all from one splitmix64 stream per case, seeded from the command line):
//   validate   random and corrupted candidate records: the library's tm_validate and
//              the oracle's or_validate must agree on the result code and the final
//              shape; valid small candidates also run through the oracle's per-point
//              evaluators (maps, chain tables, stencil and node-level volumes, matmul
//              tiles), and through tm_transpose_target (its output must validate);
//   bytes      records of random bytes: both validators must agree;
//   enumerate  tm_enumerate_factorizations against or_enum_factorizations (code,
//              count, rows), with small output capacities;
//   decompose  tm_decompose_argmin / tm_greedy_grid / tm_workload_greedy against the
//              oracle's, and tm_decompose_argmin_transpose on random inputs;
//   parse      tm_parse_index_task_map on mutated mapper texts (the corpus file given
//              on the command line, one mapper per NUL-terminated record): any result
//              code is allowed, a translated candidate must validate.
// Exit status 0 when every check holds; a sanitizer report aborts the run.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "taskmap.h"

extern "C" {
int or_validate(const void* c, int32_t* final_shape, int32_t* final_rank);
int or_proc_map(const void* c, int32_t* out, int64_t len);
int or_chain_table(const void* c, int32_t* out, int64_t cap, int64_t* count);
int or_stencil_cost(const void* c, const void* st, int64_t* out4);
int or_stencil_node_cost(const void* c, const void* st, int64_t* out4);
int or_matmul_cost(const void* c, int64_t tile_bytes, int64_t* per_proc, int64_t* out7);
int or_enum_factorizations(int64_t P, int32_t k, int32_t* out, int64_t cap, int64_t* count);
int or_decompose_argmin(int64_t P, int32_t k, const int64_t* extent, const int32_t* halo, int32_t* out_f);
int or_greedy_grid(int64_t P, int32_t k, int32_t* out_f);
int or_workload_greedy(int64_t P, int32_t k, const int64_t* extent, int32_t* out_f);
int or_sizeof_candidate(void);
}

namespace {

struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    int64_t range(int64_t lo, int64_t hi) {  // inclusive
        return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1));
    }
    bool chance(int pct) { return range(0, 99) < pct; }
};

int g_fail = 0;
long g_checks = 0;
long g_valid = 0, g_parsed = 0;  // candidates both validators accept; mappers that translate

void check(bool ok, const char* what, uint64_t seed) {
    ++g_checks;
    if (!ok && g_fail < 20) std::fprintf(stderr, "MISMATCH %s (case seed %llu)\n", what, (unsigned long long)seed);
    if (!ok) ++g_fail;
}

int64_t points_of(const tm_candidate& c) {
    int64_t p = 1;
    for (int d = 0; d < c.lrank && d < TM_MAX_LRANK; ++d) p *= c.extent[d];
    return p;
}

// A candidate that is valid more often than not: a base of merge (and sometimes
// swap), then random transformations with plausible arguments, then a projection;
// each field is corrupted now and then.
tm_candidate random_candidate(Rng& r) {
    tm_candidate c;
    std::memset(&c, 0, sizeof(c));
    c.lrank = (int32_t)r.range(1, 4);
    if (r.chance(3)) c.lrank = (int32_t)r.range(-1, 6);
    c.nodes = (int32_t)r.range(1, 12);
    c.gpus_per_node = (int32_t)(1 << r.range(0, 3));
    if (r.chance(3)) c.nodes = (int32_t)r.range(-2, 1 << 25);
    const int lr = c.lrank >= 1 && c.lrank <= 4 ? c.lrank : 2;
    for (int d = 0; d < lr; ++d) c.extent[d] = r.range(1, 12);
    if (r.chance(3)) c.extent[r.range(0, 3)] = r.chance(50) ? r.range(-3, 0) : (int64_t(1) << r.range(20, 42));
    std::vector<int64_t> shape = {c.nodes, c.gpus_per_node};
    int nops = 0;
    auto push = [&](int kind, int a, int b) {
        if (nops >= TM_MAX_OPS) return;
        tm_op& o = c.ops[nops++];
        o.kind = kind;
        o.a = a;
        o.b = b;
    };
    if (r.chance(50)) {
        push(TM_SWAP, 0, 1);
        std::swap(shape[0], shape[1]);
    }
    push(TM_MERGE, 0, 1);
    shape = {shape[0] * shape[1]};
    const int extra = (int)r.range(0, 5);
    for (int t = 0; t < extra; ++t) {
        const int rank = (int)shape.size();
        const int kind = (int)r.range(1, 5);
        if (kind == TM_DECOMPOSE) {
            const int i = (int)r.range(0, rank - 1);
            const int k = (int)r.range(1, 4);
            int64_t rest = shape[i];
            tm_op o{};
            o.kind = TM_DECOMPOSE;
            o.a = i;
            o.nf = k;
            for (int m = 0; m < k; ++m) {
                int64_t f = 1;
                if (m == k - 1) {
                    f = rest;
                } else {
                    for (int64_t dv = r.range(1, 8); dv >= 1; --dv)
                        if (rest % dv == 0) {
                            f = dv;
                            break;
                        }
                }
                o.f[m] = (int32_t)f;
                rest /= f;
            }
            if (r.chance(10)) o.f[r.range(0, 3)] = (int32_t)r.range(-1, 9);
            if (nops < TM_MAX_OPS) c.ops[nops++] = o;
            std::vector<int64_t> ns(shape.begin(), shape.begin() + i);
            for (int m = 0; m < k; ++m) ns.push_back(o.f[m]);
            ns.insert(ns.end(), shape.begin() + i + 1, shape.end());
            shape = ns;
        } else if (kind == TM_MERGE && rank >= 2) {
            const int p = (int)r.range(0, rank - 2), q = (int)r.range(p + 1, rank - 1);
            push(TM_MERGE, p, q);
            shape[p] *= shape[q];
            shape.erase(shape.begin() + q);
        } else if (kind == TM_SWAP && rank >= 2) {
            const int p = (int)r.range(0, rank - 1), q = (int)r.range(0, rank - 1);
            push(TM_SWAP, p, q);
            std::swap(shape[p], shape[q]);
        } else if (kind == TM_SPLIT || kind == TM_BALANCE_SPLIT) {
            const int i = (int)r.range(0, rank - 1);
            int64_t d = r.range(1, 6);
            if (kind == TM_SPLIT)
                while (shape[i] % d) --d;
            push(kind, i, (int)d);
            const int64_t rest = kind == TM_SPLIT ? shape[i] / d : (shape[i] + d - 1) / d;
            shape[i] = rest;
            shape.insert(shape.begin() + i, d);
        }
        if (shape.size() > TM_MAX_MRANK) break;
    }
    c.nops = nops;
    if (r.chance(4)) c.nops = (int32_t)r.range(-1, 9);
    if (r.chance(4) && nops > 0) {
        tm_op& o = c.ops[r.range(0, nops - 1)];
        switch (r.range(0, 3)) {
            case 0: o.kind = (int32_t)r.range(-1, 7); break;
            case 1: o.a = (int32_t)r.range(-2, 9); break;
            case 2: o.b = (int32_t)r.range(-2, 40); break;
            default: o.nf = (int32_t)r.range(-1, 6); break;
        }
    }
    const int fr = (int)std::min<size_t>(shape.size(), TM_MAX_MRANK);
    c.mrank = fr;
    if (r.chance(4)) c.mrank = (int32_t)r.range(-1, 9);
    for (int j = 0; j < TM_MAX_MRANK; ++j) {
        c.proj_src[j] = (int8_t)r.range(0, lr - 1);
        c.proj_mode[j] = (int8_t)(r.chance(25) ? TM_CYCLIC : TM_BLOCK);
    }
    if (r.chance(4)) c.proj_src[r.range(0, 7)] = (int8_t)r.range(-2, 6);
    if (r.chance(4)) c.proj_mode[r.range(0, 7)] = (int8_t)r.range(-1, 3);
    return c;
}

void run_oracle_evaluators(const tm_candidate& c, Rng& r) {
    const int64_t pts = points_of(c);
    if (pts <= 0 || pts > 4096) return;
    std::vector<int32_t> map((size_t)pts);
    or_proc_map(&c, map.data(), pts);
    int64_t cnt = 0;
    or_chain_table(&c, nullptr, 0, &cnt);
    if (cnt > 0 && cnt <= (1 << 20)) {
        std::vector<int32_t> t((size_t)cnt);
        or_chain_table(&c, t.data(), cnt, &cnt);
    }
    tm_stencil st;
    std::memset(&st, 0, sizeof(st));
    st.lrank = c.lrank;
    st.elem_bytes = 8;
    for (int d = 0; d < TM_MAX_LRANK; ++d) st.halo[d] = (int32_t)r.range(0, 4);
    int64_t out4[4];
    or_stencil_cost(&c, &st, out4);
    or_stencil_node_cost(&c, &st, out4);
    if (c.lrank == 3) {
        const int64_t P = (int64_t)c.nodes * c.gpus_per_node;
        if (P <= 4096) {
            std::vector<int64_t> per((size_t)P * 3);
            int64_t out7[7];
            or_matmul_cost(&c, 8, per.data(), out7);
        }
    }
}

void fuzz_validate(Rng& r, uint64_t seed) {
    tm_candidate c = random_candidate(r);
    int32_t s1[TM_MAX_MRANK] = {0}, s2[TM_MAX_MRANK] = {0}, r1 = -1, r2 = -1;
    const int a = tm_validate(&c, s1, &r1);
    const int b = or_validate(&c, s2, &r2);
    check(a == b, "validate: result codes", seed);
    if (a == TM_OK && b == 0) {
        ++g_valid;
        check(r1 == r2 && std::memcmp(s1, s2, sizeof(int32_t) * (size_t)r1) == 0, "validate: final shape", seed);
        run_oracle_evaluators(c, r);
        tm_candidate t;
        const int dim = (int)r.range(-1, 4), into = (int)r.range(-1, 4);
        if (tm_transpose_target(&c, dim, into, &t) == TM_OK) {
            int32_t s3[TM_MAX_MRANK], r3;
            check(tm_validate(&t, s3, &r3) == TM_OK, "transpose target validates", seed);
        }
    }
}

void fuzz_bytes(Rng& r, uint64_t seed) {
    tm_candidate c;
    unsigned char* p = reinterpret_cast<unsigned char*>(&c);
    for (size_t i = 0; i < sizeof(c); ++i) p[i] = (unsigned char)r.next();
    if (r.chance(50)) {  // keep the small fields in range now and then
        c.lrank = (int32_t)r.range(1, 4);
        c.nops = (int32_t)r.range(0, 8);
        c.mrank = (int32_t)r.range(1, 8);
    }
    int32_t s1[TM_MAX_MRANK], s2[TM_MAX_MRANK], r1, r2;
    const int a = tm_validate(&c, s1, &r1);
    const int b = or_validate(&c, s2, &r2);
    check((a == TM_OK) == (b == 0), "bytes: validity", seed);
}

void fuzz_enumerate(Rng& r, uint64_t seed) {
    int64_t P = r.range(1, 720);
    if (r.chance(5)) P = r.range(-3, 0);
    if (r.chance(5)) P = (int64_t(1) << 24) + r.range(-2, 2);
    const int32_t k = (int32_t)(r.chance(5) ? r.range(-1, 6) : r.range(1, 4));
    int64_t n1 = -1, n2 = -1;
    const int a0 = tm_enumerate_factorizations(P, k, nullptr, 0, &n1);
    const int b0 = or_enum_factorizations(P, k, nullptr, 0, &n2);
    check((a0 == TM_OK || a0 == TM_ECAPACITY) == (b0 == 0 || b0 == -3), "enumerate: validity", seed);
    if (!((a0 == TM_OK || a0 == TM_ECAPACITY) && (b0 == 0 || b0 == -3))) return;
    check(n1 == n2, "enumerate: count", seed);
    if (n1 <= 0 || n1 > 200000) return;
    const int64_t cap = r.chance(30) ? r.range(0, n1) : n1;
    std::vector<int32_t> o1((size_t)(cap * k) + 1, -7), o2((size_t)(n1 * k) + 1, -7);
    const int a = tm_enumerate_factorizations(P, k, o1.data(), cap, &n1);
    or_enum_factorizations(P, k, o2.data(), n2, &n2);
    if (cap < n2) {
        check(a == TM_ECAPACITY, "enumerate: capacity code", seed);
    } else {
        check(a == TM_OK && std::memcmp(o1.data(), o2.data(), sizeof(int32_t) * (size_t)(n2 * k)) == 0,
              "enumerate: rows", seed);
    }
    check(o1[(size_t)(cap * k)] == -7, "enumerate: no write past the capacity", seed);
}

void fuzz_decompose(Rng& r, uint64_t seed) {
    const int32_t k = (int32_t)r.range(1, 4);
    const int64_t P = r.range(1, 512);
    int64_t ext[4] = {1, 1, 1, 1};
    int32_t halo[4] = {0, 0, 0, 0};
    for (int d = 0; d < k; ++d) {
        ext[d] = r.range(1, 2000);
        halo[d] = (int32_t)r.range(0, 5);
    }
    int32_t f1[4] = {0}, f2[4] = {0};
    const int a = tm_decompose_argmin(P, k, ext, halo, f1), b = or_decompose_argmin(P, k, ext, halo, f2);
    check(a == b && (a != TM_OK || std::memcmp(f1, f2, sizeof(int32_t) * (size_t)k) == 0), "decompose argmin",
          seed);
    int32_t g1[4] = {0}, g2[4] = {0};
    const int c1 = tm_greedy_grid(P, k, g1), c2 = or_greedy_grid(P, k, g2);
    check(c1 == c2 && (c1 != TM_OK || std::memcmp(g1, g2, sizeof(int32_t) * (size_t)k) == 0), "greedy grid", seed);
    int32_t w1[4] = {0}, w2[4] = {0};
    const int d1 = tm_workload_greedy(P, k, ext, w1), d2 = or_workload_greedy(P, k, ext, w2);
    check(d1 == d2 && (d1 != TM_OK || std::memcmp(w1, w2, sizeof(int32_t) * (size_t)k) == 0), "workload greedy",
          seed);
    int32_t t1[4];
    const int m = (int)r.range(0, (1 << k) - 1);
    const int e = tm_decompose_argmin_transpose(P, k, ext, halo, m, t1);
    check(e == TM_OK || e == TM_EINVAL || e == TM_EOVERFLOW, "decompose with transposes: code", seed);
    if (m == 0 && e == TM_OK && a == TM_OK)
        check(std::memcmp(t1, f1, sizeof(int32_t) * (size_t)k) == 0, "decompose with no transposes", seed);
}

const char* kTokens[] = {"(", ")", "[", "]", ",", ":", ".", "*", "/", "//", "%", "+", "-", "=", "\n", "    ",
                         "#", "def", "return", "Task", "Tuple", "t", "m", "p", "ip", "ispace", "ipoint", "size",
                         "Machine(GPU)", "Machine", "GPU", "merge", "split", "swap", "balance_split", "decompose",
                         "IndexTaskMap", "0", "1", "2", "-1", "99999999999999999999", "[:-1]", "*(", "t.ipoint",
                         "m.size", "Region * * GPU FBMEM", "\t", "'", "\"", "\\", "\x01", "\xff"};

std::string mutate(const std::string& src, Rng& r) {
    std::string s = src;
    const int edits = (int)r.range(1, 6);
    for (int e = 0; e < edits; ++e) {
        const size_t n = s.size();
        const size_t at = n ? (size_t)r.range(0, (int64_t)n) : 0;
        switch (r.range(0, 5)) {
            case 0:  // flip a byte
                if (n) s[(size_t)r.range(0, (int64_t)n - 1)] = (char)r.range(1, 255);
                break;
            case 1: {  // delete a span
                const size_t len = (size_t)r.range(1, 12);
                if (at < n) s.erase(at, std::min(len, n - at));
                break;
            }
            case 2: {  // duplicate a span
                if (!n) break;
                const size_t a0 = (size_t)r.range(0, (int64_t)n - 1);
                const size_t len = std::min<size_t>((size_t)r.range(1, 24), n - a0);
                s.insert(at, s.substr(a0, len));
                break;
            }
            case 3:  // truncate
                s.resize(at);
                break;
            case 4:  // insert a token
                s.insert(at, kTokens[r.range(0, (int64_t)(sizeof(kTokens) / sizeof(kTokens[0])) - 1)]);
                break;
            default: {  // replace a digit run by another number
                for (size_t i = at; i < s.size(); ++i)
                    if (s[i] >= '0' && s[i] <= '9') {
                        s[i] = (char)('0' + r.range(0, 9));
                        break;
                    }
                break;
            }
        }
    }
    return s;
}

void fuzz_parse(Rng& r, uint64_t seed, const std::vector<std::string>& corpus) {
    std::string src;
    bool intact = false;
    if (corpus.empty() || r.chance(5)) {
        const int n = (int)r.range(0, 60);
        for (int i = 0; i < n; ++i) src += kTokens[r.range(0, (int64_t)(sizeof(kTokens) / sizeof(kTokens[0])) - 1)];
    } else {
        src = corpus[(size_t)r.range(0, (int64_t)corpus.size() - 1)];
        intact = r.chance(10);
        if (!intact) src = mutate(src, r);
    }
    const char* tasks[] = {"stencil_step", "cannon_tiles", "t3", "x", "anything", ""};
    const int32_t lrank = intact ? 2 : (int32_t)r.range(1, 4);  // the corpus mappers are 2-D
    int64_t ext[4];
    for (int d = 0; d < 4; ++d) ext[d] = r.range(1, 300);
    int32_t halo[4];
    for (int d = 0; d < 4; ++d) halo[d] = (int32_t)r.range(0, 3);
    const int32_t nodes = (int32_t)r.range(1, 16), gpus = (int32_t)(1 << r.range(0, 3));
    tm_candidate out;
    const int rc = tm_parse_index_task_map(src.c_str(), tasks[r.range(0, 5)], lrank, ext, nodes, gpus,
                                           r.chance(50) ? halo : nullptr, &out);
    check(rc == TM_OK || rc == TM_EINVAL || rc == TM_EOVERFLOW || rc == TM_ENOTSUP, "parse: result code", seed);
    if (rc == TM_OK) {
        ++g_parsed;
        int32_t s[TM_MAX_MRANK], fr;
        check(tm_validate(&out, s, &fr) == TM_OK, "parse: translated candidate validates", seed);
    }
}

std::vector<std::string> read_corpus(const char* path) {
    std::vector<std::string> out;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    std::string cur;
    int ch;
    while ((ch = std::fgetc(f)) != EOF) {
        if (ch == 0) {
            out.push_back(cur);
            cur.clear();
        } else {
            cur.push_back((char)ch);
        }
    }
    std::fclose(f);
    if (!cur.empty()) out.push_back(cur);
    return out;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s SEED CASES [CORPUS]\n", argv[0]);
        return 2;
    }
    if (or_sizeof_candidate() != (int)sizeof(tm_candidate)) {
        std::fprintf(stderr, "candidate layouts differ\n");
        return 2;
    }
    const uint64_t seed = std::strtoull(argv[1], nullptr, 10);
    const long cases = std::strtol(argv[2], nullptr, 10);
    const std::vector<std::string> corpus = argc > 3 ? read_corpus(argv[3]) : std::vector<std::string>{};
    long per_kind[5] = {0, 0, 0, 0, 0};
    for (long i = 0; i < cases; ++i) {
        const uint64_t cs = seed * 1000003ULL + (uint64_t)i;
        Rng r{cs};
        const int kind = (int)(i % 5);
        ++per_kind[kind];
        switch (kind) {
            case 0: fuzz_validate(r, cs); break;
            case 1: fuzz_bytes(r, cs); break;
            case 2: fuzz_enumerate(r, cs); break;
            case 3: fuzz_decompose(r, cs); break;
            default: fuzz_parse(r, cs, corpus); break;
        }
    }
    std::printf("cases %ld (validate %ld, bytes %ld, enumerate %ld, decompose %ld, parse %ld), checks %ld, "
                "mismatches %d, corpus %zu, valid %ld, translated %ld\n",
                cases, per_kind[0], per_kind[1], per_kind[2], per_kind[3], per_kind[4], g_checks, g_fail,
                corpus.size(), g_valid, g_parsed);
    return g_fail == 0 ? 0 : 1;
}
