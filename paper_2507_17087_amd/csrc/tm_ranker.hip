// tm_ranker.hip -- learned ranker kernels (gfx950): descriptor features, a 3-layer
// BF16 MLP (MFMA v_mfma_f32_16x16x32_bf16, FP32 accumulation) inference / forward /
// backward, Adam, the chain statistics and block-model estimates of a ranked
// search's second stage, per-segment k-smallest selection, and the on-device gather
// of the survivors for exact re-evaluation.
//
// MFMA fragment layout used throughout (16x16x32, one wave): lane l holds row
// (l % 16) of A and column (l % 16) of B, eight consecutive k values starting at
// 8 * (l / 16); the result holds rows 4 * (l / 16) + r (r = 0..3) of column l % 16.
#include <hip/hip_runtime.h>

#include "tm_chain.h"
#include "tm_internal.h"
#include "tm_ranker.h"

namespace tmk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma16(u16x8 a, u16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
}

// ------------------------------------------------------------------ features

__device__ __forceinline__ float lg2(double x) { return (float)log2(x); }

// Per-candidate chain statistics (the second stage of a ranked search):
//   cross[0..8)   per final dim j: fraction of adjacent coordinate pairs (a, a+e_j)
//                 whose owners sit on different nodes (0 for a candidate whose
//                 launch dims are each block-projected onto one final dim: its
//                 estimate does not use them);
//   cross[8..16)  the same for different processors;
//   est[0..2)     block-model estimate of the ghost cells and of the inter-node
//                 ones.  When every launch dim is projected (block) onto exactly one
//                 final dim, each cell boundary b along a launch dim is seen by the
//                 min(h, b) + min(h, l - b) cells within the halo of it, times the
//                 area of the face (product of the block widths of the other dims),
//                 counted where the owners (or nodes) on the two sides differ --
//                 exact for bijective chains whose blocks are at least h wide.
//                 Otherwise: per launch dim, the (cell, distinct foreign coordinate)
//                 pairs along it times the other extents times the crossing fraction.
// One workgroup per candidate; owners of all final coordinates staged in LDS, sized
// for the batch's largest volume (volumes above kCrossMax give zeros).
constexpr int kCrossMax = 16384;
constexpr int kStatsStage = 1024;     // launch dims up to this extent have their contributions staged in LDS
constexpr int kStatsSmallVol = 2048;  // owner-table words of the first (small-candidate) launch
constexpr int kStatsTableCap = 4096;  // block-table entries per table (simple candidates)

__device__ __forceinline__ int64_t block_first(int64_t a, int64_t S, int64_t l) { return div_nn(a * l + S - 1, S); }

// Block-model terms of final coordinate v (digits a) for a candidate whose launch
// dims are each projected (block) onto one final dim: along every dim j where v
// starts a non-empty block (a_j >= 1), the boundary b = that block's first cell is
// seen by the min(h, b) + min(h, l - b) cells within the halo of it, times the area
// of the face (the product of the other dims' block widths), counted where the
// owners (or nodes) of v and of the cell before b differ.  TAB: block bounds from
// the LDS tables, else worked out.
template <bool TAB>
__device__ __forceinline__ void boundary_terms(int32_t v, const int32_t (&a)[kMaxMrankCross], int fr,
                                               const int32_t (&fs)[kMaxMrankCross],
                                               const int32_t (&fst)[kMaxMrankCross],
                                               const int32_t (&toff)[TM_MAX_LRANK], const int32_t (&hj)[TM_MAX_LRANK],
                                               const int64_t (&lj)[TM_MAX_LRANK], const int32_t* bft,
                                               const int32_t* aLt, const int32_t* key, int gb, double& tot,
                                               double& inter) {
    int64_t bf0[TM_MAX_LRANK];
    double wd[TM_MAX_LRANK];
#pragma unroll
    for (int j = 0; j < TM_MAX_LRANK; ++j) {
        int64_t b0 = 0, b1 = 1;
        if (j < fr) {
            b0 = TAB ? bft[toff[j] + a[j]] : block_first(a[j], fs[j], lj[j]);
            b1 = TAB ? bft[toff[j] + a[j] + 1] : block_first(a[j] + 1, fs[j], lj[j]);
        }
        bf0[j] = b0;
        wd[j] = (double)(b1 - b0);
    }
    const int32_t kv = key[v];
#pragma unroll
    for (int j = 0; j < TM_MAX_LRANK; ++j) {
        if (j >= fr || a[j] == 0 || hj[j] == 0) continue;
        const int64_t b = bf0[j], l = lj[j];
        if (b >= l || wd[j] <= 0.0) continue;  // empty block
        double face = 1;
#pragma unroll
        for (int jj = 0; jj < TM_MAX_LRANK; ++jj)
            if (jj != j && jj < fr) face *= wd[jj];
        const int64_t h = hj[j];
        const double w = (double)((h < b ? h : b) + (h < l - b ? h : l - b));
        const int32_t aL = TAB ? aLt[toff[j] + a[j]] : (int32_t)div_nn((b - 1) * fs[j], l);
        const int32_t kl = key[v - (a[j] - aL) * fst[j]];
        if (kl != kv) tot += w * face;
        if ((kl >> gb) != (kv >> gb)) inter += w * face;
    }
}

__global__ __launch_bounds__(256) void k_chain_stats(const DevCand* __restrict__ cands,
                                                     const int64_t* __restrict__ idx, int64_t n,
                                                     const int32_t* __restrict__ halo, float* __restrict__ cross,
                                                     double* __restrict__ est, int32_t vmin, int32_t vmax,
                                                     int32_t vcap) {
    __shared__ DevCand sc;
    // dynamic LDS: the owner keys (vcap words, the largest volume of this launch),
    // then a region that holds either, for a simple candidate, its block tables
    // (per final dim and block a = 0..S: the block's first cell; and the block
    // holding the cell before it), tcap entries each -- the sum over dims of S + 1 is
    // at most the volume plus twice the rank -- or, otherwise, a launch dim's
    // coordinate contributions (kStatsStage entries)
    extern __shared__ __attribute__((aligned(16))) int32_t key[];
    const int32_t tcap = vcap + 16 < kStatsTableCap ? vcap + 16 : kStatsTableCap;
    int32_t* bft = key + ((vcap + 3) & ~3);
    int32_t* aLt = bft + tcap;
    int32_t* s_ct = bft;
    __shared__ int32_t red[kMaxMrankCross][4][2];  // per final dim and wave: node and owner changes
    __shared__ double dred[4][2];
    __shared__ float s_cross[2 * kMaxMrankCross];  // this candidate's crossing fractions
    __shared__ float s_rt[kRecipSlots];             // reciprocals of the inverse chain's divisors
    const int nw = blockDim.x >> 6;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        // entry i: candidate idx[i] (skipped when negative), or i without idx
        const int64_t ci = idx ? wave_uniform64(idx[i]) : i;
        if (ci < 0) continue;
        // this launch takes the candidates of volume in (vmin, vmax]; the one whose
        // vmax is kCrossMax also writes the zeros of those above it
        const int32_t v0 = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)cands[ci].vol);
        if (v0 > kCrossMax && vmax == kCrossMax) {
            if (threadIdx.x < 2 * kMaxMrankCross) cross[i * 2 * kMaxMrankCross + threadIdx.x] = 0.f;
            if (threadIdx.x < 2) est[i * 2 + threadIdx.x] = 0.0;
            continue;
        }
        if (v0 <= vmin || v0 > vmax) continue;
        lds_sync(nw);
        stage_cand(&sc, &cands[ci]);
        lds_sync(nw);
        op_reciprocals(sc, s_rt, threadIdx.x, blockDim.x);
        lds_sync(nw);
        const int32_t vol = sc.vol;
        const int K = wave_uniform(sc.lrank), gb = wave_uniform(sc.gbits), fr = wave_uniform(sc.frank);
        const int nj = fr < kMaxMrankCross ? fr : kMaxMrankCross;
        const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
        // is every launch dim projected (block) onto exactly one final dim?
        bool simple = fr == K;
        uint32_t seen = 0;
        for (int j = 0; j < fr; ++j) {
            const int d = sc.proj_src[j];
            simple = simple && sc.proj_mode[j] == TM_BLOCK && !((seen >> d) & 1u);
            seen |= 1u << d;
        }
        // the final dims' extents and strides; with simple projections, each one's
        // launch extent and halo and the offset of its block tables
        int32_t fs[kMaxMrankCross], fst[kMaxMrankCross], toff[TM_MAX_LRANK], hj[TM_MAX_LRANK];
        float rfs[kMaxMrankCross];
        int64_t lj[TM_MAX_LRANK];
#pragma unroll
        for (int j = 0; j < kMaxMrankCross; ++j) {
            fs[j] = j < fr ? wave_uniform(sc.fshape[j]) : 1;
            fst[j] = j < fr ? wave_uniform(sc.fstride[j]) : 0;
            rfs[j] = j < fr ? s_rt[kRecipFinal + j] : 1.0f;
        }
        int32_t off = 0;
#pragma unroll
        for (int j = 0; j < TM_MAX_LRANK; ++j) {
            const int d = j < fr ? wave_uniform(sc.proj_src[j]) : 0;
            toff[j] = off;
            off += j < fr ? fs[j] + 1 : 0;
            hj[j] = j < fr ? wave_uniform(halo[d]) : 0;
            lj[j] = j < fr ? wave_uniform64(sc.extent[d]) : 1;
        }
        owner_keys_sized(sc, s_rt, key, 0, 0, vol, -1, tid, blockDim.x);
        // the block tables fit when the blocks are few and the extents below 2^31
        bool tab = simple && off <= tcap;
#pragma unroll
        for (int j = 0; j < TM_MAX_LRANK; ++j) tab = tab && lj[j] < INT32_MAX;
        if (tab) {
            // per final dim: block_first of every block a (0..S) and, for a >= 1, the
            // block holding the cell before it
            for (int j = 0; j < fr; ++j) {
                const int64_t S = wave_uniform(sc.fshape[j]);
                const int64_t l = sc.extent[sc.proj_src[j]];
                int32_t o = 0;
                for (int jj = 0; jj < j; ++jj) o += wave_uniform(sc.fshape[jj]) + 1;
                for (int32_t aa = tid; aa <= (int32_t)S; aa += blockDim.x) {
                    const int64_t b = block_first(aa, S, l);
                    bft[o + aa] = (int32_t)b;
                    aLt[o + aa] = (aa >= 1 && b >= 1) ? (int32_t)div_nn((b - 1) * S, l) : 0;
                }
            }
        }
        lds_sync(nw);  // owner keys and block tables ready
        // one pass over the final coordinates: without simple projections, per final
        // dim j, the adjacent pairs (v, v + e_j) and how many of them change owner /
        // node (the crossing fractions, which only that estimate uses); with simple
        // projections the block-model estimate: every v that starts
        // a non-empty block along j (a_j >= 1) is a cell boundary b, seen by the
        // min(h, b) + min(h, l - b) cells within the halo of it times the area of the
        // face (the product of the other dims' block widths), counted where the owners
        // (or nodes) of v and of the cell before b differ -- exact for bijective chains
        // whose blocks are at least h wide.
        // per final dim: owner changes << 16 | node changes (each at most the volume,
        // below 2^16, also summed over a wave); the number of pairs is known
        int32_t ch[kMaxMrankCross];
#pragma unroll
        for (int j = 0; j < kMaxMrankCross; ++j) ch[j] = 0;
        double tot = 0, inter = 0;
        const bool need_cross = !simple;
        for (int32_t v = tid; v < vol && (need_cross || tab); v += blockDim.x) {
            int32_t a[kMaxMrankCross];
            uint32_t rem = (uint32_t)v;
#pragma unroll
            for (int j = kMaxMrankCross - 1; j >= 0; --j) {
                const uint32_t q = j < fr ? div24(rem, (uint32_t)fs[j], rfs[j]) : rem;
                a[j] = j < fr ? (int32_t)(rem - __umul24(q, (uint32_t)fs[j])) : 0;
                rem = q;
            }
            if (need_cross) {
                const int32_t kv = key[v];
#pragma unroll
                for (int j = 0; j < kMaxMrankCross; ++j) {
                    if (j < nj && a[j] < fs[j] - 1) {
                        const int32_t kn = key[v + fst[j]];
                        ch[j] += ((kn != kv) << 16) | ((kn >> gb) != (kv >> gb));
                    }
                }
            }
            if (tab) boundary_terms<true>(v, a, fr, fs, fst, toff, hj, lj, bft, aLt, key, gb, tot, inter);
        }
        // the counts summed within each wave by shuffles, then over the waves
#pragma unroll
        for (int j = 0; j < kMaxMrankCross; ++j) {
            if (j < nj && need_cross) {
#pragma unroll
                for (int o2 = 32; o2 > 0; o2 >>= 1) ch[j] += __shfl_xor(ch[j], o2, 64);
                if (lane == 0) {
                    red[j][wv][0] = ch[j] & 0xffff;
                    red[j][wv][1] = ch[j] >> 16;
                }
            }
        }
        if (simple && !tab) {  // the block tables did not fit: block bounds worked out per cell
            for (int32_t v = tid; v < vol; v += blockDim.x) {
                int32_t a[kMaxMrankCross];
                uint32_t rem = (uint32_t)v;
#pragma unroll
                for (int j = kMaxMrankCross - 1; j >= 0; --j) {
                    const uint32_t q = j < fr ? rem / (uint32_t)fs[j] : rem;
                    a[j] = j < fr ? (int32_t)(rem - __umul24(q, (uint32_t)fs[j])) : 0;
                    rem = q;
                }
                boundary_terms<false>(v, a, fr, fs, fst, toff, hj, lj, bft, aLt, key, gb, tot, inter);
            }
        }
        lds_sync(nw);
        if (tid < kMaxMrankCross) {
            const int j = tid;
            float fn = 0.f, fp = 0.f;
            if (j < nj && need_cross) {
                // pairs (v, v + e_j): the coordinates with a_j < S_j - 1
                const int32_t Sj = sc.fshape[j];
                const int pairs = (Sj - 1) * (vol / Sj);
                int dn = 0, dp = 0;
                for (int w = 0; w < nwv; ++w) {
                    dn += red[j][w][0];
                    dp += red[j][w][1];
                }
                const float inv = pairs ? 1.f / (float)pairs : 0.f;
                fn = (float)dn * inv;
                fp = (float)dp * inv;
            }
            cross[i * 2 * kMaxMrankCross + j] = fn;
            cross[i * 2 * kMaxMrankCross + kMaxMrankCross + j] = fp;
            s_cross[j] = fn;
            s_cross[kMaxMrankCross + j] = fp;
        }
        lds_sync(nw);
        if (!simple) {
            // per launch dim, the (cell, distinct foreign coordinate) pairs along it
            // times the other extents times the crossing fraction
            for (int d = 0; d < K; ++d) {
                const int64_t l = sc.extent[d];
                const int h = halo[d];
                double part = 0;
                if (h > 0 && l <= 65536) {
                    const bool staged = l <= kStatsStage;  // uniform
                    if (staged) {
                        for (int32_t x = threadIdx.x; x < (int32_t)l; x += blockDim.x) s_ct[x] = coord_value(sc, d, x);
                        lds_sync(nw);
                    }
                    for (int64_t x = threadIdx.x; x < l; x += blockDim.x) {
                        const int32_t val = staged ? s_ct[x] : coord_value(sc, d, x);
                        int32_t found[2 * kMaxHalo];
                        int cnt = 0;
                        for (int sft = 1; sft <= h && sft <= kMaxHalo; ++sft)
                            for (int dir = 0; dir < 2; ++dir) {
                                const int64_t xx = dir ? x + sft : x - sft;
                                if (xx < 0 || xx >= l) continue;
                                const int32_t dv = (staged ? s_ct[xx] : coord_value(sc, d, xx)) - val;
                                bool seen = dv == 0;
                                for (int i = 0; i < cnt; ++i) seen = seen || found[i] == dv;
                                if (!seen) found[cnt++] = dv;
                            }
                        part += cnt;
                    }
                    if (staged) lds_sync(nw);  // the next dim rewrites s_ct
                }
                float cn = 0.f, cp = 0.f;
                for (int j = 0; j < sc.frank && j < kMaxMrankCross; ++j)
                    if (sc.proj_src[j] == d) {
                        cn = fmaxf(cn, s_cross[j]);
                        cp = fmaxf(cp, s_cross[kMaxMrankCross + j]);
                    }
                double pts = 1;
                for (int dd = 0; dd < K; ++dd)
                    if (dd != d) pts *= (double)sc.extent[dd];
                tot += part * pts * cp;
                inter += part * pts * cn;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            tot += __shfl_xor(tot, o, 64);
            inter += __shfl_xor(inter, o, 64);
        }
        if (lane == 0) {
            dred[wv][0] = tot;
            dred[wv][1] = inter;
        }
        lds_sync(nw);
        if (threadIdx.x < 2) {
            double e = 0;
            for (int w = 0; w < nwv; ++w) e += dred[w][threadIdx.x];
            est[i * 2 + threadIdx.x] = e;
        }
    }
}

// The descriptor fields the features read, fetched with 16-byte loads: each group
// below starts at a 16-byte aligned offset of DevCand (checked here), so a thread
// issues 15 vector loads per candidate instead of one load per field.
static_assert(offsetof(DevCand, lrank) == 0 && offsetof(DevCand, nops) == 4 && offsetof(DevCand, nodes) == 8 &&
                  offsetof(DevCand, gpus) == 12 && offsetof(DevCand, gbits) == 16 && offsetof(DevCand, frank) == 20,
              "descriptor header");
static_assert(offsetof(DevCand, extent) == 32, "extents");
static_assert(offsetof(DevCand, fshape) % 16 == 0 && TM_MAX_MRANK == 8, "final shape");
static_assert(offsetof(DevCand, proj_mode) == offsetof(DevCand, proj_src) + 8 && offsetof(DevCand, proj_src) % 16 == 0,
              "projections");
static_assert(offsetof(DevCand, op_kind) % 16 == 0 && offsetof(DevCand, op_a) % 16 == 0 &&
                  offsetof(DevCand, op_b) % 16 == 0 && offsetof(DevCand, op_nf) % 16 == 0 &&
                  offsetof(DevCand, op_f) % 16 == 0 && TM_MAX_OPS == 8 && TM_MAX_LRANK == 4,
              "ops");

struct FeatDesc {
    int k, nops, nodes, gpus, gbits, fr;
    int64_t ext[TM_MAX_LRANK];
    int32_t fsh[TM_MAX_MRANK];
    int32_t psrc[TM_MAX_MRANK], pmode[TM_MAX_MRANK];
    int32_t kind[TM_MAX_OPS], opa[4], opb[TM_MAX_OPS];
    int tdec, nf;
    int32_t F[TM_MAX_LRANK];  // the factors of the first decompose (1 past nf)
};

__device__ __forceinline__ FeatDesc load_feat_desc(const DevCand* c) {
    const int4* q = reinterpret_cast<const int4*>(c);
    auto at = [&](size_t off) { return q[off / 16]; };
    FeatDesc d;
    const int4 h0 = at(0), h1 = at(16);
    d.k = h0.x, d.nops = h0.y, d.nodes = h0.z, d.gpus = h0.w, d.gbits = h1.x, d.fr = h1.y;
    const int4 e0 = at(32), e1 = at(48);
    d.ext[0] = (int64_t)(((uint64_t)(uint32_t)e0.y << 32) | (uint32_t)e0.x);
    d.ext[1] = (int64_t)(((uint64_t)(uint32_t)e0.w << 32) | (uint32_t)e0.z);
    d.ext[2] = (int64_t)(((uint64_t)(uint32_t)e1.y << 32) | (uint32_t)e1.x);
    d.ext[3] = (int64_t)(((uint64_t)(uint32_t)e1.w << 32) | (uint32_t)e1.z);
    const int4 f0 = at(offsetof(DevCand, fshape)), f1 = at(offsetof(DevCand, fshape) + 16);
    const int32_t fs[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
    const int4 pj = at(offsetof(DevCand, proj_src));
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        d.fsh[j] = fs[j];
        d.psrc[j] = (int32_t)(int8_t)(((j < 4 ? pj.x : pj.y) >> (8 * (j & 3))) & 0xff);
        d.pmode[j] = (int32_t)(int8_t)(((j < 4 ? pj.z : pj.w) >> (8 * (j & 3))) & 0xff);
    }
    const int4 k0 = at(offsetof(DevCand, op_kind)), k1 = at(offsetof(DevCand, op_kind) + 16);
    const int4 b0 = at(offsetof(DevCand, op_b)), b1 = at(offsetof(DevCand, op_b) + 16);
    const int4 n0 = at(offsetof(DevCand, op_nf)), n1 = at(offsetof(DevCand, op_nf) + 16);
    const int4 a0 = at(offsetof(DevCand, op_a));
    const int32_t kk[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
    const int32_t bb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
    const int32_t nn[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
    d.opa[0] = a0.x, d.opa[1] = a0.y, d.opa[2] = a0.z, d.opa[3] = a0.w;
    d.tdec = -1;
    d.nf = 0;
#pragma unroll
    for (int t = TM_MAX_OPS - 1; t >= 0; --t) {
        d.kind[t] = kk[t];
        d.opb[t] = bb[t];
        if (t < d.nops && kk[t] == TM_DECOMPOSE) {
            d.tdec = t;
            d.nf = nn[t];
        }
    }
    const int4 fv = q[(offsetof(DevCand, op_f) + 16 * (d.tdec >= 0 ? d.tdec : 0)) / 16];
    d.F[0] = 0 < d.nf ? fv.x : 1;
    d.F[1] = 1 < d.nf ? fv.y : 1;
    d.F[2] = 2 < d.nf ? fv.z : 1;
    d.F[3] = 3 < d.nf ? fv.w : 1;
    return d;
}

// Descriptor estimate of the ghost cells, from the shapes alone: if every change of
// the final coordinates projected from a launch dim changes the processor (a
// bijective chain), the processor changes along launch dim d at l - 1 coordinate
// boundaries when a final dim of size > 1 is projected onto it cyclically, and
// otherwise at the interior block starts of its block-projected final dims (at most
// the sum of their sizes less one each, and at most l - 1); every boundary puts 2h
// cells of each cross-section into the halo.  Exact for bijective chains with one
// final dim per launch dim whose blocks are at least h wide.
__device__ __forceinline__ double descriptor_estimate(const FeatDesc& c, const int32_t* __restrict__ halo) {
    double cells = 0;
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) {
        if (d >= c.k) continue;
        const int64_t l = c.ext[d];
        int64_t nb = 0;
        bool cyc = false;
#pragma unroll
        for (int j = 0; j < TM_MAX_MRANK; ++j) {
            if (j >= c.fr || c.psrc[j] != d) continue;
            if (c.pmode[j] != TM_BLOCK) cyc = cyc || c.fsh[j] > 1;
            else nb += c.fsh[j] - 1;
        }
        nb = cyc ? l - 1 : (nb < l - 1 ? nb : l - 1);
        double face = 1;
#pragma unroll
        for (int e = 0; e < TM_MAX_LRANK; ++e)
            if (e < c.k && e != d) face *= (double)c.ext[e];
        cells += 2.0 * halo[d] * (double)nb * face;
    }
    return cells;
}

// log2 in fp32 for the features other than the estimate's (they are compared with
// the fp64 reference at 1e-5 and stored in bf16)
__device__ __forceinline__ float lg2f(float x) { return log2f(x); }

// One thread per candidate; writes kFeat bf16 values (row of X, eight 16-byte
// stores), the descriptor estimate (est[2i]; est[2i+1] = 0: no inter-node base)
// and, when feat_f32 is given, the features in fp32.
__global__ __launch_bounds__(256) void k_features(const DevCand* __restrict__ cands, int64_t n,
                                                  const int32_t* __restrict__ halo, double* __restrict__ est,
                                                  uint16_t* __restrict__ X, float* __restrict__ feat_f32) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const FeatDesc c = load_feat_desc(cands + i);
    // every index into f and the small arrays below is static once the loops are
    // unrolled (bounded by the ABI's maxima, the candidate's counts as predicates), so
    // all of them live in registers
    float f[kFeat];
#pragma unroll
    for (int t = 0; t < kFeat; ++t) f[t] = 0.f;
    const int k = c.k, fr = c.fr, nops = c.nops, nf = c.nf;
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) f[d] = d == k - 1 ? 1.f : 0.f;
    // blocks per launch dim: the product of the final extents it projects onto
    double blocks[TM_MAX_LRANK] = {1, 1, 1, 1};
#pragma unroll
    for (int j = 0; j < TM_MAX_MRANK; ++j) {
        if (j < fr) {
            const int src = c.psrc[j];
            const double sh = (double)c.fsh[j];
#pragma unroll
            for (int d = 0; d < TM_MAX_LRANK; ++d) blocks[d] *= src == d ? sh : 1.0;
        }
    }
    int32_t hl[TM_MAX_LRANK];
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) hl[d] = d < k ? halo[d] : 0;
    double vol_f = 0;
#pragma unroll
    for (int d = 0; d < TM_MAX_LRANK; ++d) {
        if (d < k) {
            const double l = (double)c.ext[d];
            const float ll = lg2f((float)l), lb = lg2f((float)blocks[d]);
            f[4 + d] = ll / 10.f;
            f[15 + d] = lb / 9.f;
            f[19 + d] = (ll - lb) / 10.f;
            if (d < nf) vol_f += 2.0 * hl[d] * (c.F[d] - 1.0) / l;
            f[54 + d] = hl[d] / 4.f;
        }
    }
    f[8] = lg2f((float)c.nodes) / 6.f;
    f[9] = lg2f((float)c.gpus) / 3.f;
    f[10] = lg2f((float)c.nodes * (float)c.gpus) / 9.f;
#pragma unroll
    for (int m = 0; m < TM_MAX_LRANK; ++m)
        if (m < nf) f[11 + m] = lg2f((float)c.F[m]) / 9.f;
    f[24] = lg2f((float)(1.0 + vol_f)) / 4.f;
#pragma unroll
    for (int t = 0; t < TM_MAX_OPS; ++t) {
        if (t < nops) {
            const int kd = c.kind[t];
#pragma unroll
            for (int q = 0; q < 5; ++q) f[25 + q] += kd == q + 1 ? 0.25f : 0.f;
            if (t < 6) {
                f[30 + t] = kd / 5.f;
                if (t < 3) f[39 + t] = c.opa[t] / 8.f;
                f[42 + t] = kd == TM_DECOMPOSE ? 0.f : lg2f(1.f + (float)c.opb[t]) / 9.f;
            }
        }
    }
    f[48] = (nops > 0 && c.kind[0] == TM_SWAP) ? 1.f : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j < fr) f[49 + j] = c.pmode[j] ? 1.f : 0.f;
    f[53] = fr / 8.f;
    f[58] = c.gbits / 3.f;
    f[59] = 1.f;
    // the descriptor estimate of the ghost cells in the log space of the target (the
    // inter-node head has no base: feature kBaseFeat[1] stays 0)
    const double e0 = descriptor_estimate(c, hl);
    *reinterpret_cast<double2*>(est + i * 2) = make_double2(e0, 0.0);
    f[kBaseFeat[0]] = lg2(1.0 + e0) / kBaseScale;
    uint4* row = reinterpret_cast<uint4*>(X + i * kFeat);
#pragma unroll
    for (int t = 0; t < kFeat / 8; ++t) {
        uint4 w;
        w.x = (uint32_t)f2bf(f[8 * t]) | ((uint32_t)f2bf(f[8 * t + 1]) << 16);
        w.y = (uint32_t)f2bf(f[8 * t + 2]) | ((uint32_t)f2bf(f[8 * t + 3]) << 16);
        w.z = (uint32_t)f2bf(f[8 * t + 4]) | ((uint32_t)f2bf(f[8 * t + 5]) << 16);
        w.w = (uint32_t)f2bf(f[8 * t + 6]) | ((uint32_t)f2bf(f[8 * t + 7]) << 16);
        row[t] = w;
    }
    if (feat_f32) {
        float4* fo = reinterpret_cast<float4*>(feat_f32 + i * kFeat);
#pragma unroll
        for (int t = 0; t < kFeat / 4; ++t) fo[t] = make_float4(f[4 * t], f[4 * t + 1], f[4 * t + 2], f[4 * t + 3]);
    }
}

// ------------------------------------------------------------------ fused forward
//
// A workgroup of the forward pass (8 waves) takes 64 rows.  Activations stay in LDS
// (bf16, padded row stride); wave w computes output columns [32w, 32w + 32) of
// each hidden layer as 4 x 2 MFMA tiles, reading weight fragments straight from
// the transposed bf16 weights Wt[n][k] (16 contiguous bytes per lane).  Measured on
// 1M rows: 8 waves of 32 columns 0.58 ms, 4 of 64 columns 0.63 ms, 16 of 16
// columns 0.72 ms, 128-row workgroups 0.70 ms.  The tiles are computed
// transposed (weights as the first operand), so a lane ends with four consecutive
// columns of one row: the epilogue (bias, ReLU, round to bf16) writes them to LDS
// as one 8-byte store; optionally the activations are stored for the backward pass.
// The head (256 -> 2) is one more MFMA tile per wave against the two weight columns
// staged in LDS (the other 14 columns zero): bf16 products summed in fp32.

constexpr int kRowsFwd = 64;    // rows per workgroup of the backward-data kernel
constexpr int kRowsMlp = 64;    // rows per workgroup of the forward pass
constexpr int kMlpThreads = 512;
constexpr int kMlpNB = kWidth / 16 / (kMlpThreads / 64);  // 16-column blocks per wave
constexpr int kMlpInferCus = 256;  // persistent inference workgroups (one per CU)
constexpr int kLdsStride = kWidth + 8;  // bf16 elements per LDS row (breaks bank aliasing)

template <int KIN, int NB>
__device__ __forceinline__ void layer_fwd(const uint16_t* __restrict__ in_lds, uint16_t* __restrict__ out_lds,
                                          const uint16_t* __restrict__ Wt, const float* __restrict__ bias,
                                          int lane, int cbase) {
    f32x4 acc[4][NB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    // two k-steps in flight
#pragma unroll 2
    for (int k0 = 0; k0 < KIN; k0 += 32) {
        u16x8 bf[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int ncol = cbase + b * 16 + r16;
            bf[b] = *reinterpret_cast<const u16x8*>(Wt + (size_t)ncol * KIN + k0 + kq);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const u16x8 af = *reinterpret_cast<const u16x8*>(in_lds + (a * 16 + r16) * kLdsStride + k0 + kq);
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[a][b] = mfma16(bf[b], af, acc[a][b]);
        }
    }
    // acc[a][b][r]: row a*16 + r16, column cbase + b*16 + (lane>>4)*4 + r
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int col0 = cbase + b * 16 + (lane >> 4) * 4;
        const float b0 = bias[col0], b1 = bias[col0 + 1], b2 = bias[col0 + 2], b3 = bias[col0 + 3];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int row = a * 16 + r16;
            uint2 w;
            w.x = (uint32_t)f2bf(fmaxf(acc[a][b][0] + b0, 0.f)) | ((uint32_t)f2bf(fmaxf(acc[a][b][1] + b1, 0.f)) << 16);
            w.y = (uint32_t)f2bf(fmaxf(acc[a][b][2] + b2, 0.f)) | ((uint32_t)f2bf(fmaxf(acc[a][b][3] + b3, 0.f)) << 16);
            *reinterpret_cast<uint2*>(out_lds + row * kLdsStride + col0) = w;
        }
    }
}

__device__ __forceinline__ void store_act(const uint16_t* __restrict__ lds_act, uint16_t* __restrict__ g,
                                          int64_t row0, int64_t n, int tid) {
    // kRowsMlp rows x 256 bf16: each thread moves 8 bf16 per step
    for (int i = tid; i < kRowsMlp * (kWidth / 8); i += kMlpThreads) {
        const int r = i / (kWidth / 8), c8 = (i % (kWidth / 8)) * 8;
        if (row0 + r < n)
            *reinterpret_cast<u16x8*>(g + (row0 + r) * kWidth + c8) =
                *reinterpret_cast<const u16x8*>(lds_act + r * kLdsStride + c8);
    }
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(const uint16_t* __restrict__ X, int64_t n,
                                                             const RankerWeights W, float* __restrict__ Y,
                                                             uint16_t* __restrict__ H1, uint16_t* __restrict__ H2,
                                                             uint16_t* __restrict__ H3) {
    __shared__ __attribute__((aligned(16))) uint16_t sa[kRowsMlp * kLdsStride];
    __shared__ __attribute__((aligned(16))) uint16_t sb[kRowsMlp * kLdsStride];
    __shared__ __attribute__((aligned(16))) uint16_t s_w4[kOut * kWidth];  // head weights, transposed
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int cbase = wid * kMlpNB * 16;  // this wave's output columns
    for (int i = tid; i < kOut * kWidth; i += kMlpThreads) s_w4[(i % kOut) * kWidth + i / kOut] = W.w4[i];
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const float hb = r16 < kOut ? W.b4[r16] : 0.f;
    for (int64_t row0 = (int64_t)blockIdx.x * kRowsMlp; row0 < n; row0 += (int64_t)gridDim.x * kRowsMlp) {
        __syncthreads();
        // X tile -> sa (kRowsMlp x 64 bf16), zero rows past n
        for (int i = tid; i < kRowsMlp * (kFeat / 8); i += kMlpThreads) {
            const int r = i / (kFeat / 8), c8 = (i % (kFeat / 8)) * 8;
            u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (row0 + r < n) v = *reinterpret_cast<const u16x8*>(X + (row0 + r) * kFeat + c8);
            *reinterpret_cast<u16x8*>(sa + r * kLdsStride + c8) = v;
        }
        __syncthreads();
        layer_fwd<kFeat, kMlpNB>(sa, sb, W.w1t, W.b1, lane, cbase);
        __syncthreads();
        if (H1) store_act(sb, H1, row0, n, tid);
        layer_fwd<kWidth, kMlpNB>(sb, sa, W.w2t, W.b2, lane, cbase);
        __syncthreads();
        if (H2) store_act(sa, H2, row0, n, tid);
        layer_fwd<kWidth, kMlpNB>(sa, sb, W.w3t, W.b3, lane, cbase);
        __syncthreads();
        if (H3) store_act(sb, H3, row0, n, tid);
        // head: wave w < 4 takes rows 16w..16w+15; B columns 0, 1 are the two heads
        if (wid < kRowsMlp / 16) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int k0 = 0; k0 < kWidth; k0 += 32) {
                const u16x8 af = *reinterpret_cast<const u16x8*>(sb + (wid * 16 + r16) * kLdsStride + k0 + kq);
                const u16x8 wf = *reinterpret_cast<const u16x8*>(s_w4 + (r16 < kOut ? r16 : 0) * kWidth + k0 + kq);
                acc = mfma16(af, r16 < kOut ? wf : zero, acc);
            }
            // acc[r]: row wid*16 + (lane>>4)*4 + r, output r16
            if (r16 < kOut) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + wid * 16 + (lane >> 4) * 4 + r;
                    if (row < n) Y[row * kOut + r16] = acc[r] + hb;
                }
            }
        }
    }
}

// Inference over many rows (no activations stored): a persistent workgroup per CU
// keeps its waves' weight fragments in registers for every row tile it takes, so
// the weights are read from L2 once per workgroup instead of once per tile.
template <int KIN>
__device__ __forceinline__ void load_wfrag(u16x8 (&wf)[KIN / 32][kMlpNB], const uint16_t* __restrict__ Wt, int lane,
                                           int cbase) {
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int ks = 0; ks < KIN / 32; ++ks)
#pragma unroll
        for (int b = 0; b < kMlpNB; ++b)
            wf[ks][b] = *reinterpret_cast<const u16x8*>(Wt + (size_t)(cbase + b * 16 + r16) * KIN + ks * 32 + kq);
}

template <int KIN>
__device__ __forceinline__ void layer_reg(const uint16_t* __restrict__ in_lds, uint16_t* __restrict__ out_lds,
                                          const u16x8 (&wf)[KIN / 32][kMlpNB], const float* __restrict__ bias,
                                          int lane, int cbase) {
    f32x4 acc[4][kMlpNB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < kMlpNB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int ks = 0; ks < KIN / 32; ++ks) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const u16x8 af = *reinterpret_cast<const u16x8*>(in_lds + (a * 16 + r16) * kLdsStride + ks * 32 + kq);
#pragma unroll
            for (int b = 0; b < kMlpNB; ++b) acc[a][b] = mfma16(wf[ks][b], af, acc[a][b]);
        }
    }
#pragma unroll
    for (int b = 0; b < kMlpNB; ++b) {
        const int col0 = cbase + b * 16 + (lane >> 4) * 4;
        const float b0 = bias[col0], b1 = bias[col0 + 1], b2 = bias[col0 + 2], b3 = bias[col0 + 3];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int row = a * 16 + r16;
            uint2 w;
            w.x = (uint32_t)f2bf(fmaxf(acc[a][b][0] + b0, 0.f)) | ((uint32_t)f2bf(fmaxf(acc[a][b][1] + b1, 0.f)) << 16);
            w.y = (uint32_t)f2bf(fmaxf(acc[a][b][2] + b2, 0.f)) | ((uint32_t)f2bf(fmaxf(acc[a][b][3] + b3, 0.f)) << 16);
            *reinterpret_cast<uint2*>(out_lds + row * kLdsStride + col0) = w;
        }
    }
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_infer(const uint16_t* __restrict__ X, int64_t n,
                                                           const RankerWeights W, float* __restrict__ Y) {
    __shared__ __attribute__((aligned(16))) uint16_t sa[kRowsMlp * kLdsStride];
    __shared__ __attribute__((aligned(16))) uint16_t sb[kRowsMlp * kLdsStride];
    __shared__ __attribute__((aligned(16))) uint16_t s_w4[kOut * kWidth];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int cbase = wid * kMlpNB * 16;
    for (int i = tid; i < kOut * kWidth; i += kMlpThreads) s_w4[(i % kOut) * kWidth + i / kOut] = W.w4[i];
    u16x8 w1[kFeat / 32][kMlpNB], w2[kWidth / 32][kMlpNB], w3[kWidth / 32][kMlpNB];
    load_wfrag<kFeat>(w1, W.w1t, lane, cbase);
    load_wfrag<kWidth>(w2, W.w2t, lane, cbase);
    load_wfrag<kWidth>(w3, W.w3t, lane, cbase);
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const float hb = r16 < kOut ? W.b4[r16] : 0.f;
    // one 16-byte piece of a 64 x 64 feature tile per thread; the next tile's piece is
    // loaded while the current tile runs through the layers
    static_assert(kRowsMlp * (kFeat / 8) == kMlpThreads, "one feature piece per thread");
    const int xr = tid / (kFeat / 8), xc = (tid % (kFeat / 8)) * 8;
    const int64_t step = (int64_t)gridDim.x * kRowsMlp;
    auto x_piece = [&](int64_t r0) {
        u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (r0 + xr < n) v = *reinterpret_cast<const u16x8*>(X + (r0 + xr) * kFeat + xc);
        return v;
    };
    *reinterpret_cast<u16x8*>(sa + xr * kLdsStride + xc) = x_piece((int64_t)blockIdx.x * kRowsMlp);
    for (int64_t row0 = (int64_t)blockIdx.x * kRowsMlp; row0 < n; row0 += step) {
        __syncthreads();  // this tile's features in sa; the previous head is done with sb
        const u16x8 xn = x_piece(row0 + step);
        layer_reg<kFeat>(sa, sb, w1, W.b1, lane, cbase);
        __syncthreads();
        layer_reg<kWidth>(sb, sa, w2, W.b2, lane, cbase);
        __syncthreads();
        layer_reg<kWidth>(sa, sb, w3, W.b3, lane, cbase);
        __syncthreads();  // sa is free: the next tile's features go in
        *reinterpret_cast<u16x8*>(sa + xr * kLdsStride + xc) = xn;
        if (wid < kRowsMlp / 16) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int k0 = 0; k0 < kWidth; k0 += 32) {
                const u16x8 af = *reinterpret_cast<const u16x8*>(sb + (wid * 16 + r16) * kLdsStride + k0 + kq);
                const u16x8 wf = *reinterpret_cast<const u16x8*>(s_w4 + (r16 < kOut ? r16 : 0) * kWidth + k0 + kq);
                acc = mfma16(af, r16 < kOut ? wf : zero, acc);
            }
            if (r16 < kOut) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + wid * 16 + (lane >> 4) * 4 + r;
                    if (row < n) Y[row * kOut + r16] = acc[r] + hb;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ backward pieces

// dY = scale_h * (Y - T) (per head weights already in scale), and the head's input
// gradient dH3 = (dY W4^T) * [H3 > 0], bf16.
__global__ __launch_bounds__(256) void k_head_backward(const float* __restrict__ Y, const float* __restrict__ Tg,
                                                       int64_t n, float s0, float s1, const RankerWeights W,
                                                       const uint16_t* __restrict__ H3, float* __restrict__ dY,
                                                       uint16_t* __restrict__ dH3) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * kWidth) return;
    const int64_t r = idx / kWidth;
    const int k = (int)(idx % kWidth);
    const float d0 = s0 * (Y[r * kOut] - Tg[r * kOut]);
    const float d1 = s1 * (Y[r * kOut + 1] - Tg[r * kOut + 1]);
    if (k == 0) {
        dY[r * kOut] = d0;
        dY[r * kOut + 1] = d1;
    }
    const float g = d0 * bf2f(W.w4[k * kOut]) + d1 * bf2f(W.w4[k * kOut + 1]);
    dH3[idx] = bf2f(H3[idx]) > 0.f ? f2bf(g) : (uint16_t)0;
}

// dIn = (dOut M) * [Act > 0] where the layer computed Out = In Wf: M = Wf^T, so
// B-fragments come from Wf stored row-major [kin][kout] (k = kout contiguous).
// 64 rows per workgroup, KOUT = 256 reduction, output columns KIN.
template <int KIN>
__global__ __launch_bounds__(256) void k_backward_data(const uint16_t* __restrict__ dOut, int64_t n,
                                                       const uint16_t* __restrict__ Wf,
                                                       const uint16_t* __restrict__ Act,
                                                       uint16_t* __restrict__ dIn) {
    __shared__ __attribute__((aligned(16))) uint16_t sa[kRowsFwd * kLdsStride];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    constexpr int NT = KIN / 64;  // column tiles of 16 per wave
    for (int64_t row0 = (int64_t)blockIdx.x * kRowsFwd; row0 < n; row0 += (int64_t)gridDim.x * kRowsFwd) {
        __syncthreads();
        for (int i = tid; i < kRowsFwd * (kWidth / 8); i += 256) {
            const int r = i / (kWidth / 8), c8 = (i % (kWidth / 8)) * 8;
            u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (row0 + r < n) v = *reinterpret_cast<const u16x8*>(dOut + (row0 + r) * kWidth + c8);
            *reinterpret_cast<u16x8*>(sa + r * kLdsStride + c8) = v;
        }
        __syncthreads();
        f32x4 acc[4][NT];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < kWidth; k0 += 32) {
            u16x8 bf[NT];
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int ncol = wid * (KIN / 4) + b * 16 + r16;
                bf[b] = *reinterpret_cast<const u16x8*>(Wf + (size_t)ncol * kWidth + k0 + kq);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const u16x8 af = *reinterpret_cast<const u16x8*>(sa + (a * 16 + r16) * kLdsStride + k0 + kq);
#pragma unroll
                for (int b = 0; b < NT; ++b) acc[a][b] = mfma16(af, bf[b], acc[a][b]);
            }
        }
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const int col = wid * (KIN / 4) + b * 16 + r16;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + a * 16 + (lane >> 4) * 4 + r;
                    if (row < n) {
                        const bool on = Act ? bf2f(Act[row * KIN + col]) > 0.f : true;
                        dIn[row * KIN + col] = on ? f2bf(acc[a][b][r]) : (uint16_t)0;
                    }
                }
        }
    }
}

// Weight gradient partials: P[split][KIN][KOUT] = In[rows of split]^T dOut[rows].
// Workgroup = (64 x 64 output tile, split).  Chunks of 32 rows are staged in LDS
// transposed (k-major) so that both MFMA operands read 16 contiguous bytes.
template <int KIN>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ In, const uint16_t* __restrict__ dOut,
                                               int64_t n, int64_t rows_per_split, float* __restrict__ P) {
    __shared__ __attribute__((aligned(16))) uint16_t sI[64][40];  // [kin][row] (32 rows + pad)
    __shared__ __attribute__((aligned(16))) uint16_t sO[64][40];  // [kout][row]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tiles_n = kWidth / 64;
    const int ti = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;  // output tile (kin, kout)
    const int split = blockIdx.y;
    const int64_t ra = split * rows_per_split;
    const int64_t rb = ra + rows_per_split < n ? ra + rows_per_split : n;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const int wa = wid >> 1, wb = wid & 1;  // wave's 32 x 32 quadrant
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t r0 = ra; r0 < rb; r0 += 32) {
        __syncthreads();
        // 32 rows x 64 columns of each operand, transposed into LDS
        for (int i = tid; i < 32 * 64; i += 256) {
            const int rr = i / 64, cc = i % 64;
            const int64_t row = r0 + rr;
            uint16_t vi = 0, vo = 0;
            if (row < rb) {
                vi = In[row * KIN + ti * 64 + cc];
                vo = dOut[row * kWidth + tn * 64 + cc];
            }
            sI[cc][rr] = vi;
            sO[cc][rr] = vo;
        }
        __syncthreads();
        const u16x8 a0 = *reinterpret_cast<const u16x8*>(&sI[wa * 32 + r16][kq]);
        const u16x8 a1 = *reinterpret_cast<const u16x8*>(&sI[wa * 32 + 16 + r16][kq]);
        const u16x8 b0 = *reinterpret_cast<const u16x8*>(&sO[wb * 32 + r16][kq]);
        const u16x8 b1 = *reinterpret_cast<const u16x8*>(&sO[wb * 32 + 16 + r16][kq]);
        acc[0][0] = mfma16(a0, b0, acc[0][0]);
        acc[0][1] = mfma16(a0, b1, acc[0][1]);
        acc[1][0] = mfma16(a1, b0, acc[1][0]);
        acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
    float* out = P + (size_t)split * KIN * kWidth;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * 64 + wa * 32 + a * 16 + (lane >> 4) * 4 + r;
                const int col = tn * 64 + wb * 32 + b * 16 + r16;
                out[row * kWidth + col] = acc[a][b][r];
            }
}

// Column sums of a bf16 [n x N] matrix per split (bias gradients), fp32 partials.
__global__ __launch_bounds__(256) void k_colsum(const uint16_t* __restrict__ A, int64_t n, int N,
                                                int64_t rows_per_split, float* __restrict__ P) {
    const int split = blockIdx.y;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= N) return;
    const int64_t ra = split * rows_per_split;
    const int64_t rb = ra + rows_per_split < n ? ra + rows_per_split : n;
    // eight partial sums (eight loads in flight), combined in a fixed order
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int64_t r = ra;
    for (; r + 8 <= rb; r += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += bf2f(A[(r + u) * N + col]);
    }
    for (; r < rb; ++r) acc[0] += bf2f(A[r * N + col]);
    P[(size_t)split * N + col] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Head gradients: dW4[k][h] = sum_r H3[r][k] dY[r][h], db4[h] = sum_r dY[r][h].
__global__ __launch_bounds__(256) void k_head_wgrad(const uint16_t* __restrict__ H3, const float* __restrict__ dY,
                                                    int64_t n, int64_t rows_per_split, float* __restrict__ P) {
    const int split = blockIdx.y;
    const int t = threadIdx.x;  // k index
    const int64_t ra = split * rows_per_split;
    const int64_t rb = ra + rows_per_split < n ? ra + rows_per_split : n;
    // four partial sums of each (four rows' loads in flight), combined in a fixed order
    float s0[4] = {0.f, 0.f, 0.f, 0.f}, s1[4] = {0.f, 0.f, 0.f, 0.f};
    float c0[4] = {0.f, 0.f, 0.f, 0.f}, c1[4] = {0.f, 0.f, 0.f, 0.f};
    int64_t r = ra;
    for (; r + 4 <= rb; r += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float h = bf2f(H3[(r + u) * kWidth + t]);
            const float y0 = dY[(r + u) * kOut], y1 = dY[(r + u) * kOut + 1];
            s0[u] += h * y0;
            s1[u] += h * y1;
            c0[u] += y0;
            c1[u] += y1;
        }
    }
    for (; r < rb; ++r) {
        const float h = bf2f(H3[r * kWidth + t]);
        const float y0 = dY[r * kOut], y1 = dY[r * kOut + 1];
        s0[0] += h * y0;
        s1[0] += h * y1;
        c0[0] += y0;
        c1[0] += y1;
    }
    const float t0 = (s0[0] + s0[1]) + (s0[2] + s0[3]), t1 = (s1[0] + s1[1]) + (s1[2] + s1[3]);
    const float b0 = (c0[0] + c0[1]) + (c0[2] + c0[3]), b1 = (c1[0] + c1[1]) + (c1[2] + c1[3]);
    float* o = P + (size_t)split * (kWidth * kOut + kOut);
    o[t * kOut] = t0;
    o[t * kOut + 1] = t1;
    if (t == 0) {
        o[kWidth * kOut] = b0;
        o[kWidth * kOut + 1] = b1;
    }
}

// Sum split partials (fixed order: deterministic) into dst[count].
__global__ __launch_bounds__(256) void k_reduce_splits(const float* __restrict__ P, int splits, int64_t count,
                                                       float* __restrict__ dst) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    // four partial sums (four loads in flight), combined in a fixed order
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int sp = 0;
    for (; sp + 4 <= splits; sp += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += P[(size_t)(sp + u) * count + i];
    }
    for (; sp < splits; ++sp) acc[0] += P[(size_t)sp * count + i];
    dst[i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Adam on the fp32 master copy; refreshes the bf16 copies (row-major and
// transposed) of the matrices.  Parameter layout: see RankerLayout.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t count,
                                              float lr, float b1, float b2, float eps, float c1, float c2,
                                              const RankerWeights W) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    publish_param(i, pi, W);
}

// Refresh all bf16 copies from the fp32 master (after loading or setting params).
__global__ __launch_bounds__(256) void k_publish(const float* __restrict__ p, int64_t count, const RankerWeights W) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    publish_param(i, p[i], W);
}

// ------------------------------------------------------------------ k smallest per segment
//
// One workgroup per segment chooses its k smallest (score, index) pairs by a radix
// select over the scores' order-preserving 32-bit keys: three passes of 11, 11 and
// 10 bits, each a histogram in LDS of the keys that share the digits found so far,
// give the k-th smallest key T and how many of the k equal it; one pass in index
// order then takes every key below T and the lowest-indexed keys equal to T.  The
// chosen entries are written in index order, then -1 up to k.  Segment s is
// [seg[s], seg[s+1]), or with stride > 0 the first min(stride, seg[s+1] - seg[s])
// entries from s * stride.  margin > 0 keeps of the chosen only those scoring at
// most `margin` above the segment's best.  remap (nullable) gives the index written
// for entry e (else e).  Scores are finite or +inf.

__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

constexpr int kSelThreads = 256;
constexpr int kSelBins = 2048;  // 8 per thread

__global__ __launch_bounds__(kSelThreads) void k_select(const float* __restrict__ score,
                                                        const int64_t* __restrict__ seg, int64_t stride, int k,
                                                        float margin, const int64_t* __restrict__ remap,
                                                        int64_t* __restrict__ sel) {
    __shared__ uint32_t hist[kSelBins];
    __shared__ uint32_t wa[kSelThreads / 64], wb[kSelThreads / 64];
    __shared__ float wmin[kSelThreads / 64];
    __shared__ uint32_t s_bin, s_below;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int nwv = kSelThreads / 64;
    const int64_t s = blockIdx.x;
    const int64_t len_s = seg[s + 1] - seg[s];
    const int64_t a = stride > 0 ? s * stride : seg[s];
    const uint32_t len = (uint32_t)(stride > 0 ? (len_s < stride ? len_s : stride) : len_s);
    int64_t* out = sel + s * (int64_t)k;
    const uint64_t lt_mask = (1ull << lane) - 1;
    // the segment's best score (the margin's reference)
    float best = INFINITY;
    for (uint32_t i = tid; i < len; i += kSelThreads) best = fminf(best, score[a + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = fminf(best, __shfl_xor(best, o, 64));
    if (lane == 0) wmin[wv] = best;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < nwv; ++w) best = fminf(best, wmin[w]);
    // the k-th smallest key T; rem = how many of the chosen have key T
    const bool all = len <= (uint32_t)k;
    uint32_t prefix = 0, pmask = 0, rem = all ? len : (uint32_t)k;
    if (!all) {
        for (int pass = 0; pass < 3; ++pass) {
            const int shift = pass == 0 ? 21 : (pass == 1 ? 10 : 0);
            const uint32_t dmask = pass == 2 ? 0x3ffu : 0x7ffu;
            for (int b = tid; b < kSelBins; b += kSelThreads) hist[b] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < len; i += kSelThreads) {
                const uint32_t kk = order_key(score[a + i]);
                if ((kk & pmask) == prefix) atomicAdd(&hist[(kk >> shift) & dmask], 1u);
            }
            __syncthreads();
            uint32_t c[8], tsum = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                c[q] = hist[tid * 8 + q];
                tsum += c[q];
            }
            uint32_t incl = tsum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = __shfl_up(incl, o, 64);
                incl += lane >= o ? u : 0u;
            }
            if (lane == 63) wa[wv] = incl;
            __syncthreads();
            uint32_t run = incl - tsum;
            for (int w = 0; w < wv; ++w) run += wa[w];
            // exactly one bin has run < rem <= run + count
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (run < rem && run + c[q] >= rem) {
                    s_bin = (uint32_t)(tid * 8 + q);
                    s_below = run;
                }
                run += c[q];
            }
            __syncthreads();
            prefix |= s_bin << shift;
            pmask |= dmask << shift;
            rem -= s_below;
            __syncthreads();  // s_bin, s_below and hist are rewritten by the next pass
        }
    }
    // in index order: keys below T, then the first rem keys equal to T
    const uint32_t T = prefix;
    uint32_t seen_eq = 0, written = 0;
    for (uint32_t i0 = 0; i0 < len; i0 += kSelThreads) {
        const uint32_t i = i0 + tid;
        bool in = false, eq = false;
        float sv = INFINITY;
        if (i < len) {
            sv = score[a + i];
            const uint32_t kk = order_key(sv);
            in = all || kk < T;
            eq = !all && kk == T;
        }
        const uint64_t beq = __ballot(eq);
        if (lane == 0) wa[wv] = (uint32_t)__popcll(beq);
        __syncthreads();
        uint32_t eq_rank = (uint32_t)__popcll(beq & lt_mask), chunk_eq = 0;
#pragma unroll
        for (int w = 0; w < nwv; ++w) {
            eq_rank += w < wv ? wa[w] : 0u;
            chunk_eq += wa[w];
        }
        const bool take = (in || (eq && seen_eq + eq_rank < rem)) && (margin <= 0.f || sv <= best + margin);
        const uint64_t bt = __ballot(take);
        if (lane == 0) wb[wv] = (uint32_t)__popcll(bt);
        __syncthreads();
        uint32_t pos = (uint32_t)__popcll(bt & lt_mask), chunk_t = 0;
#pragma unroll
        for (int w = 0; w < nwv; ++w) {
            pos += w < wv ? wb[w] : 0u;
            chunk_t += wb[w];
        }
        if (take && written + pos < (uint32_t)k) out[written + pos] = remap ? remap[a + i] : a + i;
        written += chunk_t;
        seen_eq += chunk_eq;
        __syncthreads();  // wa, wb are rewritten by the next chunk
    }
    for (int64_t r = (int64_t)written + tid; r < k; r += kSelThreads) out[r] = -1;
}

// Ranking score: predicted log2(1 + bytes) + lambda * predicted log2(1 + inter-node
// bytes), each = estimate base (the same fp32 value training used) + un-standardised
// residual head; without Y the estimates alone; +inf when that is not finite.
__global__ void k_combine(const float* __restrict__ Y, const double* __restrict__ est, int64_t n, float mu0,
                          float s0, float mu1, float s1, float lambda, float* __restrict__ s) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b0 = kBaseScale * (lg2(1.0 + est[i * 2]) / kBaseScale);
    const float b1 = kBaseScale * (lg2(1.0 + est[i * 2 + 1]) / kBaseScale);
    const float p0 = Y ? b0 + mu0 + s0 * Y[i * kOut] : b0, p1 = Y ? b1 + mu1 + s1 * Y[i * kOut + 1] : b1;
    const float v = p0 + lambda * p1;
    // a non-finite score (diverged or corrupt parameters) ranks last, by index, so
    // such candidates stay selectable and every instance keeps its survivors
    s[i] = __builtin_isfinite(v) ? v : INFINITY;
}

// ------------------------------------------------------------------ survivors

// Builds the sub-batch of selected candidates on the device, in three launches.
// k_gather_sizes reads each selected candidate's table words and counting items;
// k_gather (one workgroup, 4 consecutive entries per thread) lays out their tables
// and work items by prefix sums over the selection (per-thread sums, wave scans,
// then the waves' totals), writes the sub-batch entry j of
// every selected candidate -- map[j] = its original index and the three fields that
// change (arena_off, item_first, citems) -- the sub-batch segments and header;
// k_gather_copy then copies the rest of the descriptors, word by word across the
// grid.  sel[s] < 0 entries are skipped; seg_out gives the sub-batch segments.
constexpr int kDescWords = (int)(sizeof(DevCand) / 4);
constexpr int kArenaWord = (int)(offsetof(DevCand, arena_off) / 4);
constexpr int kItemWord = (int)(offsetof(DevCand, item_first) / 4);
constexpr int kCitemsWord = (int)(offsetof(DevCand, citems) / 4);
static_assert(sizeof(DevCand) % 4 == 0, "descriptor copied as words");

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        v += lane >= o ? u : 0;
    }
    return v;
}

// Sizes of the selected candidates, one thread per entry: sizes[2s] = the table
// words of candidate sel[s] (-1 when sel[s] < 0), sizes[2s+1] = its counting items.
__global__ void k_gather_sizes(const DevCand* __restrict__ cands, const int64_t* __restrict__ sel, int64_t nsel,
                               int64_t cells_per_item, int64_t* __restrict__ sizes) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= nsel) return;
    const int64_t ci = sel[s];
    int64_t w = -1, it = 0;
    if (ci >= 0) {
        const DevCand& c = cands[ci];
        w = c.words;
        it = count_items(c, cells_per_item);
    }
    sizes[2 * s] = w;
    sizes[2 * s + 1] = it;
}

constexpr int kGatherPer = 4;  // consecutive entries per thread of k_gather

__global__ __launch_bounds__(1024) void k_gather(const int64_t* __restrict__ sel, const int64_t* __restrict__ sizes,
                                                 int64_t nsel, int k, DevCand* __restrict__ sub,
                                                 int64_t* __restrict__ map, int64_t* __restrict__ seg_out,
                                                 DevHeader* __restrict__ hdr, const DevHeader* __restrict__ proto) {
    __shared__ int64_t s_tot[16][3];  // per wave: words, items, present
    __shared__ int64_t carry[3];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    if (tid < 3) carry[tid] = 0;
    __syncthreads();
    const int64_t span = (int64_t)blockDim.x * kGatherPer;
    for (int64_t base = 0; base < nsel; base += span) {
        // this thread's entries s0 .. s0 + kGatherPer - 1: their totals, then a
        // block-wide scan of the totals, then the entries in order
        const int64_t s0 = base + (int64_t)tid * kGatherPer;
        int64_t words = 0, items = 0, present = 0;
        for (int q = 0; q < kGatherPer && s0 + q < nsel; ++q) {
            const int64_t w = sizes[2 * (s0 + q)];
            if (w >= 0) {
                words += w;
                items += sizes[2 * (s0 + q) + 1];
                ++present;
            }
        }
        const int64_t iw = wave_incl_scan(words, lane), ii = wave_incl_scan(items, lane),
                      ic = wave_incl_scan(present, lane);
        if (lane == 63) {
            s_tot[wid][0] = iw;
            s_tot[wid][1] = ii;
            s_tot[wid][2] = ic;
        }
        __syncthreads();
        int64_t pw = carry[0] + iw - words, pi = carry[1] + ii - items, pc = carry[2] + ic - present;
        for (int w = 0; w < wid; ++w) {
            pw += s_tot[w][0];
            pi += s_tot[w][1];
            pc += s_tot[w][2];
        }
        for (int q = 0; q < kGatherPer && s0 + q < nsel; ++q) {
            const int64_t s = s0 + q;
            // segment starts: first slot of each segment of k
            if (s % k == 0) seg_out[s / k] = pc;
            const int64_t w = sizes[2 * s];
            if (w >= 0) {
                const int64_t it = sizes[2 * s + 1];
                map[pc] = sel[s];
                sub[pc].arena_off = pw;
                sub[pc].item_first = pi;
                sub[pc].citems = (int32_t)it;
                pw += w;
                pi += it;
                ++pc;
            }
        }
        __syncthreads();  // every thread has read carry and s_tot
        if (tid < 3) {
            int64_t t = 0;
            for (int w = 0; w < nw; ++w) t += s_tot[w][tid];
            carry[tid] += t;
        }
        __syncthreads();
    }
    if (tid == 0) {
        seg_out[(nsel + k - 1) / k] = carry[2];
        DevHeader h = *proto;
        h.n = carry[2];
        h.total_items = carry[1];
        h.item_tab = carry[0];  // the survivors' item table follows their tables
        *hdr = h;
    }
}

__global__ __launch_bounds__(256) void k_gather_copy(const DevCand* __restrict__ cands,
                                                     const int64_t* __restrict__ map,
                                                     const DevHeader* __restrict__ hdr, DevCand* __restrict__ sub) {
    const int64_t total = hdr->n * kDescWords;
    const int32_t* src = reinterpret_cast<const int32_t*>(cands);
    int32_t* dst = reinterpret_cast<int32_t*>(sub);
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / kDescWords;
        const int w = (int)(t - j * kDescWords);
        if (w == kArenaWord || w == kArenaWord + 1 || w == kItemWord || w == kItemWord + 1 || w == kCitemsWord)
            continue;  // written by k_gather
        dst[t] = src[map[j] * kDescWords + w];
    }
}

// best[s] = map[sub_best[s] + seg[s]] (original candidate index) and its cost.
__global__ void k_map_best(const int64_t* __restrict__ sub_best, const int64_t* __restrict__ seg,
                           const int64_t* __restrict__ map, const tm_stencil_cost* __restrict__ sub_cost,
                           int64_t nseg, const int64_t* __restrict__ orig_seg, int64_t* __restrict__ best,
                           tm_stencil_cost* __restrict__ best_cost) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t b = sub_best[s];
    if (b < 0) {
        best[s] = -1;
        if (best_cost) best_cost[s] = tm_stencil_cost{-1, -1, -1, -1};
        return;
    }
    const int64_t j = seg[s] + b;
    best[s] = map[j] - orig_seg[s];
    if (best_cost) best_cost[s] = sub_cost[j];
}

// Exhaustive path: best index is already relative; copy costs out.
__global__ void k_pick_costs(const int64_t* __restrict__ best, const int64_t* __restrict__ seg,
                             const tm_stencil_cost* __restrict__ cost, int64_t nseg,
                             tm_stencil_cost* __restrict__ best_cost) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= nseg || !best_cost) return;
    best_cost[s] = best[s] < 0 ? tm_stencil_cost{-1, -1, -1, -1} : cost[seg[s] + best[s]];
}

// ------------------------------------------------------------------ launchers

hipError_t launch_features(const DevCand* cands, int64_t n, const int32_t* d_halo, double* est, uint16_t* X,
                           float* f32, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cands, n, d_halo, est, X, f32);
    return hipGetLastError();
}

hipError_t launch_chain_stats(const DevCand* cands, const int64_t* idx, int64_t n, int32_t max_vol,
                              const int32_t* d_halo, float* cross, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t g = n < 65536 ? n : 65536;
    double* est = chain_estimates(cross, n);
    // the owner table of a candidate lives in LDS: most candidates are small, so a
    // first launch with a small table (more workgroups per CU) takes the volumes up to
    // kStatsSmallVol, and a second one, sized for the batch's largest, the rest;
    // large batches of small candidates: one-wave workgroups, four times as many
    // candidates in flight per CU (each candidate's work is a few hundred keys)
    const int bs = n >= kSmallBlockBatch ? 64 : 256;
    const int32_t vtop = std::max(1, std::min(max_vol, kCrossMax));
    // LDS words: the keys, then the two block tables or a launch dim's contributions
    auto lds_bytes = [](int32_t vcap) {
        const int32_t tcap = std::min(vcap + 16, kStatsTableCap);
        return (size_t)(((vcap + 3) & ~3) + std::max(2 * tcap, kStatsStage)) * 4;
    };
    if (vtop <= kStatsSmallVol) {
        hipLaunchKernelGGL(k_chain_stats, dim3((unsigned)g), dim3(bs), lds_bytes(vtop), s, cands, idx, n, d_halo,
                           cross, est, 0, kCrossMax, vtop);
    } else {
        hipLaunchKernelGGL(k_chain_stats, dim3((unsigned)g), dim3(bs), lds_bytes(kStatsSmallVol), s, cands, idx, n,
                           d_halo, cross, est, 0, kStatsSmallVol, kStatsSmallVol);
        hipLaunchKernelGGL(k_chain_stats, dim3((unsigned)g), dim3(bs), lds_bytes(vtop), s, cands, idx, n, d_halo,
                           cross, est, kStatsSmallVol, kCrossMax, vtop);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t* X, int64_t n, const RankerWeights& W, float* Y, uint16_t* H1,
                              uint16_t* H2, uint16_t* H3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + kRowsMlp - 1) / kRowsMlp;
    if (!H1 && !H2 && !H3 && grid > 4 * kMlpInferCus) {
        // inference over many rows: persistent workgroups, weights in registers
        hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)kMlpInferCus), dim3(kMlpThreads), 0, s, X, n, W, Y);
        return hipGetLastError();
    }
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)grid), dim3(kMlpThreads), 0, s, X, n, W, Y, H1, H2, H3);
    return hipGetLastError();
}

hipError_t launch_backward(const RankerBuffers& B, const RankerWeights& W, int64_t n, float s0, float s1,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t rows_per_split = ((n + kSplits - 1) / kSplits + 31) / 32 * 32;
    const int splits = (int)((n + rows_per_split - 1) / rows_per_split);
    hipLaunchKernelGGL(k_head_backward, dim3((unsigned)((n * kWidth + 255) / 256)), dim3(256), 0, s, B.Y, B.T, n, s0,
                       s1, W, B.H3, B.dY, B.dH3);
    hipLaunchKernelGGL(k_head_wgrad, dim3(1, splits), dim3(kWidth), 0, s, B.H3, B.dY, n, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3((kWidth * kOut + kOut + 255) / 256), dim3(256), 0, s, B.part, splits,
                       (int64_t)(kWidth * kOut + kOut), B.grad + W.layout.w4);
    int64_t grid = (n + kRowsFwd - 1) / kRowsFwd;
    if (grid > 8192) grid = 8192;
    // layer 3
    hipLaunchKernelGGL(k_wgrad<kWidth>, dim3(16, splits), dim3(256), 0, s, B.H2, B.dH3, n, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3((kWidth * kWidth + 255) / 256), dim3(256), 0, s, B.part, splits,
                       (int64_t)kWidth * kWidth, B.grad + W.layout.w3);
    hipLaunchKernelGGL(k_colsum, dim3(1, splits), dim3(kWidth), 0, s, B.dH3, n, kWidth, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3(1), dim3(256), 0, s, B.part, splits, (int64_t)kWidth, B.grad + W.layout.b3);
    hipLaunchKernelGGL(k_backward_data<kWidth>, dim3((unsigned)grid), dim3(256), 0, s, B.dH3, n, W.w3, B.H2, B.dH2);
    // layer 2
    hipLaunchKernelGGL(k_wgrad<kWidth>, dim3(16, splits), dim3(256), 0, s, B.H1, B.dH2, n, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3((kWidth * kWidth + 255) / 256), dim3(256), 0, s, B.part, splits,
                       (int64_t)kWidth * kWidth, B.grad + W.layout.w2);
    hipLaunchKernelGGL(k_colsum, dim3(1, splits), dim3(kWidth), 0, s, B.dH2, n, kWidth, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3(1), dim3(256), 0, s, B.part, splits, (int64_t)kWidth, B.grad + W.layout.b2);
    hipLaunchKernelGGL(k_backward_data<kWidth>, dim3((unsigned)grid), dim3(256), 0, s, B.dH2, n, W.w2, B.H1, B.dH1);
    // layer 1
    hipLaunchKernelGGL(k_wgrad<kFeat>, dim3(4, splits), dim3(256), 0, s, B.X, B.dH1, n, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3((kFeat * kWidth + 255) / 256), dim3(256), 0, s, B.part, splits,
                       (int64_t)kFeat * kWidth, B.grad + W.layout.w1);
    hipLaunchKernelGGL(k_colsum, dim3(1, splits), dim3(kWidth), 0, s, B.dH1, n, kWidth, rows_per_split, B.part);
    hipLaunchKernelGGL(k_reduce_splits, dim3(1), dim3(256), 0, s, B.part, splits, (int64_t)kWidth, B.grad + W.layout.b1);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2,
                       float eps, int64_t t, const RankerWeights& W, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, g, m, v, count, lr, b1, b2,
                       eps, c1, c2, W);
    return hipGetLastError();
}

hipError_t launch_publish(const float* p, int64_t count, const RankerWeights& W, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, W);
    return hipGetLastError();
}

hipError_t launch_select(const float* score, const int64_t* seg, int64_t nseg, int64_t stride, int k, float margin,
                         const int64_t* remap, int64_t* sel, hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3((unsigned)nseg), dim3(kSelThreads), 0, s, score, seg, stride, k, margin, remap,
                       sel);
    return hipGetLastError();
}

hipError_t launch_combine(const float* Y, const double* est, int64_t n, const float* mu, const float* sigma,
                          float lambda, float* s, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Y, est, n, mu[0], sigma[0],
                       mu[1], sigma[1], lambda, s);
    return hipGetLastError();
}

hipError_t launch_gather(const DevCand* cands, const int64_t* sel, int64_t nsel, int k, int64_t cells_per_item,
                         DevCand* sub, int64_t* map, int64_t* seg_out, DevHeader* hdr, const DevHeader* proto,
                         int64_t* sizes, hipStream_t s) {
    if (nsel > 0)
        hipLaunchKernelGGL(k_gather_sizes, dim3((unsigned)((nsel + 255) / 256)), dim3(256), 0, s, cands, sel, nsel,
                           cells_per_item, sizes);
    hipLaunchKernelGGL(k_gather, dim3(1), dim3(1024), 0, s, sel, sizes, nsel, k, sub, map, seg_out, hdr, proto);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsel <= 0) return e;
    const int64_t blocks = (nsel * kDescWords + 255) / 256;
    hipLaunchKernelGGL(k_gather_copy, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, cands, map,
                       hdr, sub);
    return hipGetLastError();
}

hipError_t launch_map_best(const int64_t* sub_best, const int64_t* seg, const int64_t* map,
                           const tm_stencil_cost* sub_cost, int64_t nseg, const int64_t* orig_seg, int64_t* best,
                           tm_stencil_cost* best_cost, hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_best, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, s, sub_best, seg, map, sub_cost,
                       nseg, orig_seg, best, best_cost);
    return hipGetLastError();
}

hipError_t launch_pick_costs(const int64_t* best, const int64_t* seg, const tm_stencil_cost* cost, int64_t nseg,
                             tm_stencil_cost* best_cost, hipStream_t s) {
    if (nseg <= 0 || !best_cost) return hipSuccess;
    hipLaunchKernelGGL(k_pick_costs, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, s, best, seg, cost, nseg,
                       best_cost);
    return hipGetLastError();
}

}  // namespace tmk
