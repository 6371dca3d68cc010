// tm_ranker_host.cpp -- learned ranker object (parameters, Adam state, training
// loop) and the ranked search over a loaded plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
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

static uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static double unit(uint64_t& s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace tmk

using namespace tmk;

struct tm_ranker {
    RankerLayout L = ranker_layout();
    float *p = nullptr, *m = nullptr, *v = nullptr;  // fp32 master, Adam moments
    uint16_t* bf = nullptr;                          // all bf16 copies in one block
    RankerWeights W{};
    float mu[kOut] = {0, 0}, sigma[kOut] = {1, 1};   // target standardisation
    int64_t step = 0;
    // training buffers (grown on demand)
    RankerBuffers B{};
    int64_t cap_rows = 0;
    void* bufmem = nullptr;
};

namespace tmk {

static int ranker_alloc_weights(tm_ranker* r) {
    const int64_t n = r->L.count;
    TM_HIP(hipMalloc((void**)&r->p, n * 4));
    TM_HIP(hipMalloc((void**)&r->m, n * 4));
    TM_HIP(hipMalloc((void**)&r->v, n * 4));
    TM_HIP(hipMemset(r->m, 0, n * 4));
    TM_HIP(hipMemset(r->v, 0, n * 4));
    const int64_t nb = 2 * (kFeat * kWidth) + 4 * (kWidth * kWidth) + kWidth * kOut;
    TM_HIP(hipMalloc((void**)&r->bf, nb * 2));
    uint16_t* q = r->bf;
    r->W.w1 = q; q += kFeat * kWidth;
    r->W.w1t = q; q += kFeat * kWidth;
    r->W.w2 = q; q += kWidth * kWidth;
    r->W.w2t = q; q += kWidth * kWidth;
    r->W.w3 = q; q += kWidth * kWidth;
    r->W.w3t = q; q += kWidth * kWidth;
    r->W.w4 = q;
    r->W.b1 = r->p + r->L.b1;
    r->W.b2 = r->p + r->L.b2;
    r->W.b3 = r->p + r->L.b3;
    r->W.b4 = r->p + r->L.b4;
    r->W.layout = r->L;
    return TM_OK;
}

static int ranker_buffers(tm_ranker* r, int64_t rows) {
    if (rows <= r->cap_rows) return TM_OK;
    if (r->bufmem) TM_HIP(hipFree(r->bufmem));
    r->bufmem = nullptr;
    rows = std::max<int64_t>(rows, 1024);
    const size_t bf = (size_t)rows * (kFeat + 6 * kWidth) * 2;
    const size_t f32 = (size_t)rows * 3 * kOut * 4 + (size_t)r->L.count * 4 + (size_t)kSplits * kWidth * kWidth * 4;
    if (hipMalloc(&r->bufmem, bf + f32 + 1024) != hipSuccess) return set_error(TM_ENOMEM, "ranker buffers");
    char* q = (char*)r->bufmem;
    auto take = [&](size_t bytes) {
        void* p = q;
        q += (bytes + 255) & ~size_t(255);
        return p;
    };
    r->B.X = (uint16_t*)take((size_t)rows * kFeat * 2);
    r->B.H1 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.H2 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.H3 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.dH1 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.dH2 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.dH3 = (uint16_t*)take((size_t)rows * kWidth * 2);
    r->B.Y = (float*)take((size_t)rows * kOut * 4);
    r->B.T = (float*)take((size_t)rows * kOut * 4);
    r->B.dY = (float*)take((size_t)rows * kOut * 4);
    r->B.grad = (float*)take((size_t)r->L.count * 4);
    r->B.part = (float*)take((size_t)kSplits * kWidth * kWidth * 4);
    r->cap_rows = rows;
    return TM_OK;
}

// fp32 features -> bf16 rows, optionally gathered through a permutation; targets
// gathered likewise.
__global__ void k_pack_batch(const float* __restrict__ feat, const float* __restrict__ tgt,
                             const int64_t* __restrict__ perm, int64_t first, int64_t rows,
                             uint16_t* __restrict__ X, float* __restrict__ T) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= rows * kFeat) return;
    const int64_t r = i / kFeat, c = i % kFeat;
    const int64_t src = perm ? perm[first + r] : first + r;
    uint32_t u = __float_as_uint(feat[src * kFeat + c]);
    u += 0x7fffu + ((u >> 16) & 1u);
    X[i] = (uint16_t)(u >> 16);
    if (c < kOut && T && tgt) T[r * kOut + c] = tgt[src * kOut + c];
}

// Standardised targets from exact costs: t_h = (log2(1 + x_h) - mu_h) / sigma_h.
// Residual targets: log2(1 + exact bytes) minus the estimate base carried by the
// features (kBaseScale * feature kBaseFeat[h]).
__device__ __forceinline__ double residual(const tm_stencil_cost& c, const float* feat, int64_t i, int h) {
    const double x = log2(1.0 + (double)(h == 0 ? c.bytes : c.inter_bytes));
    return x - (double)(kBaseScale * feat[i * kFeat + kBaseFeat[h]]);
}

__global__ void k_targets(const tm_stencil_cost* __restrict__ cost, const float* __restrict__ feat, int64_t n,
                          float m0, float s0, float m1, float s1, float* __restrict__ T) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    T[i * kOut] = (float)((residual(cost[i], feat, i, 0) - m0) / s0);
    T[i * kOut + 1] = (float)((residual(cost[i], feat, i, 1) - m1) / s1);
}

// Per-block sums of the residual targets and their squares for both heads (fp64 partials).
__global__ __launch_bounds__(256) void k_target_moments(const tm_stencil_cost* __restrict__ cost,
                                                        const float* __restrict__ feat, int64_t n,
                                                        double* __restrict__ part) {
    __shared__ double s[4][256];
    double a0 = 0, a1 = 0, q0 = 0, q1 = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x0 = residual(cost[i], feat, i, 0), x1 = residual(cost[i], feat, i, 1);
        a0 += x0;
        a1 += x1;
        q0 += x0 * x0;
        q1 += x1 * x1;
    }
    s[0][threadIdx.x] = a0;
    s[1][threadIdx.x] = a1;
    s[2][threadIdx.x] = q0;
    s[3][threadIdx.x] = q1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 4; ++j) s[j][threadIdx.x] += s[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

// Mean squared error over rows and heads (fp64 partial sums per block).
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ Y, const float* __restrict__ T, int64_t n,
                                              double* __restrict__ part) {
    __shared__ double s[256];
    double a = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * kOut;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)Y[i] - (double)T[i];
        a += d * d;
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

static int ranker_forward_rows(tm_ranker* r, const uint16_t* X, int64_t rows, float* Y, bool keep, hipStream_t s) {
    const hipError_t e = launch_mlp_forward(X, rows, r->W, Y, keep ? r->B.H1 : nullptr, keep ? r->B.H2 : nullptr,
                                            keep ? r->B.H3 : nullptr, s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "forward: %s", hipGetErrorString(e));
    return TM_OK;
}

// Gradient of the mean squared error of one batch (rows already packed in B).
static int ranker_batch_grad(tm_ranker* r, int64_t rows, hipStream_t s) {
    int rc = ranker_forward_rows(r, r->B.X, rows, r->B.Y, true, s);
    if (rc != TM_OK) return rc;
    const float sc = 2.0f / (float)(rows * kOut);
    const hipError_t e = launch_backward(r->B, r->W, rows, sc, sc, s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "backward: %s", hipGetErrorString(e));
    return TM_OK;
}

}  // namespace tmk

extern "C" {

int tm_ranker_param_count(void) { return (int)ranker_layout().count; }
int tm_ranker_feature_count(void) { return kFeat; }

int tm_ranker_create(uint64_t seed, tm_ranker** out) {
    if (!out) return set_error(TM_EINVAL, "null output");
    *out = nullptr;
    tm_ranker* r = new (std::nothrow) tm_ranker();
    if (!r) return set_error(TM_ENOMEM, "ranker");
    int rc = ranker_alloc_weights(r);
    if (rc != TM_OK) {
        tm_ranker_destroy(r);
        return rc;
    }
    // He-normal weights (Box-Muller over splitmix64), zero biases
    std::vector<float> h((size_t)r->L.count, 0.f);
    uint64_t st = seed ^ 0x7a5b0d1e3c2f4a69ULL;
    auto fill = [&](int64_t off, int64_t fan_in, int64_t cnt) {
        const double sd = std::sqrt(2.0 / (double)fan_in);
        for (int64_t i = 0; i < cnt; ++i) {
            const double u1 = std::max(unit(st), 1e-300), u2 = unit(st);
            h[(size_t)(off + i)] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    };
    fill(r->L.w1, kFeat, kFeat * kWidth);
    fill(r->L.w2, kWidth, kWidth * kWidth);
    fill(r->L.w3, kWidth, kWidth * kWidth);
    fill(r->L.w4, kWidth, kWidth * kOut);
    if (hipMemcpy(r->p, h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        launch_publish(r->p, r->L.count, r->W, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        tm_ranker_destroy(r);
        return set_error(TM_EDEVICE, "ranker init");
    }
    *out = r;
    return TM_OK;
}

int tm_ranker_destroy(tm_ranker* r) {
    if (!r) return TM_OK;
    (void)hipDeviceSynchronize();
    if (r->p) (void)hipFree(r->p);
    if (r->m) (void)hipFree(r->m);
    if (r->v) (void)hipFree(r->v);
    if (r->bf) (void)hipFree(r->bf);
    if (r->bufmem) (void)hipFree(r->bufmem);
    delete r;
    return TM_OK;
}

int tm_ranker_get_params(tm_ranker* r, float* d_out, void* stream) {
    if (!r || !d_out) return set_error(TM_EINVAL, "null argument");
    TM_HIP(hipMemcpyAsync(d_out, r->p, r->L.count * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return TM_OK;
}

int tm_ranker_set_params(tm_ranker* r, const float* d_in, void* stream) {
    if (!r || !d_in) return set_error(TM_EINVAL, "null argument");
    TM_HIP(hipMemcpyAsync(r->p, d_in, r->L.count * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    TM_HIP(launch_publish(r->p, r->L.count, r->W, (hipStream_t)stream));
    return TM_OK;
}

int tm_ranker_get_scaling(const tm_ranker* r, float* mu_sigma) {
    if (!r || !mu_sigma) return set_error(TM_EINVAL, "null argument");
    mu_sigma[0] = r->mu[0];
    mu_sigma[1] = r->sigma[0];
    mu_sigma[2] = r->mu[1];
    mu_sigma[3] = r->sigma[1];
    return TM_OK;
}

int tm_ranker_forward(tm_ranker* r, const float* d_feat, int64_t n, float* d_out, void* stream) {
    if (!r || n < 0 || (n > 0 && (!d_feat || !d_out))) return set_error(TM_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int64_t chunk = 1 << 18;
    int rc = ranker_buffers(r, std::min<int64_t>(n, chunk));
    if (rc != TM_OK) return rc;
    for (int64_t a = 0; a < n; a += chunk) {
        const int64_t rows = std::min(chunk, n - a);
        hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)((rows * kFeat + 255) / 256)), dim3(256), 0, s, d_feat,
                           nullptr, nullptr, a, rows, r->B.X, nullptr);
        rc = ranker_forward_rows(r, r->B.X, rows, d_out + a * kOut, false, s);
        if (rc != TM_OK) return rc;
    }
    return TM_OK;
}

int tm_ranker_grad(tm_ranker* r, const float* d_feat, const float* d_target, int64_t n, float* d_grad,
                   void* stream) {
    if (!r || n <= 0 || !d_feat || !d_target || !d_grad) return set_error(TM_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int rc = ranker_buffers(r, n);
    if (rc != TM_OK) return rc;
    hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)((n * kFeat + 255) / 256)), dim3(256), 0, s, d_feat, d_target,
                       nullptr, 0, n, r->B.X, r->B.T);
    rc = ranker_batch_grad(r, n, s);
    if (rc != TM_OK) return rc;
    TM_HIP(hipMemcpyAsync(d_grad, r->B.grad, r->L.count * 4, hipMemcpyDeviceToDevice, s));
    return TM_OK;
}

int tm_ranker_train(tm_ranker* r, const float* d_feat, const tm_stencil_cost* d_cost, int64_t n, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, float* h_loss, void* stream) {
    if (!r || n <= 0 || !d_feat || !d_cost || epochs < 0 || batch < 1) return set_error(TM_EINVAL, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    // target scaling from the training set
    const int nb = 512;
    double* d_part = nullptr;
    float* d_T = nullptr;
    int64_t* d_perm = nullptr;
    TM_HIP(hipMalloc((void**)&d_part, nb * 4 * sizeof(double)));
    hipLaunchKernelGGL(k_target_moments, dim3(nb), dim3(256), 0, s, d_cost, d_feat, n, d_part);
    std::vector<double> part(nb * 4);
    TM_HIP(hipMemcpyAsync(part.data(), d_part, part.size() * 8, hipMemcpyDeviceToHost, s));
    TM_HIP(hipStreamSynchronize(s));
    double a[4] = {0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int j = 0; j < 4; ++j) a[j] += part[b * 4 + j];
    for (int h = 0; h < kOut; ++h) {
        const double mean = a[h] / n, var = std::max(a[2 + h] / n - mean * mean, 1e-12);
        r->mu[h] = (float)mean;
        r->sigma[h] = (float)std::max(std::sqrt(var), 1e-3);
    }
    int rc = TM_OK;
    if (hipMalloc((void**)&d_T, (size_t)n * kOut * 4) != hipSuccess ||
        hipMalloc((void**)&d_perm, (size_t)n * 8) != hipSuccess)
        rc = set_error(TM_ENOMEM, "training buffers");
    if (rc == TM_OK) {
        hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_cost, d_feat, n, r->mu[0],
                           r->sigma[0], r->mu[1], r->sigma[1], d_T);
        rc = ranker_buffers(r, batch);
    }
    std::vector<int64_t> perm((size_t)n);
    uint64_t st = seed ^ 0x2545F4914F6CDD1DULL;
    for (int ep = 0; ep < epochs && rc == TM_OK; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[(size_t)i], perm[(size_t)(splitmix(st) % (uint64_t)(i + 1))]);
        if (hipMemcpyAsync(d_perm, perm.data(), (size_t)n * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = set_error(TM_EDEVICE, "permutation upload");
            break;
        }
        double loss_sum = 0;
        int64_t loss_rows = 0;
        for (int64_t first = 0; first + batch <= n || (first < n && first == 0); first += batch) {
            const int64_t rows = std::min<int64_t>(batch, n - first);
            hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)((rows * kFeat + 255) / 256)), dim3(256), 0, s, d_feat,
                               d_T, d_perm, first, rows, r->B.X, r->B.T);
            rc = ranker_batch_grad(r, rows, s);
            if (rc != TM_OK) break;
            ++r->step;
            // cosine decay over the run
            const double prog = (double)(ep * ((n + batch - 1) / batch) + first / batch) /
                                (double)std::max<int64_t>(1, epochs * ((n + batch - 1) / batch));
            const float lr_t = (float)(lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(3.141592653589793 * prog))));
            if (launch_adam(r->p, r->B.grad, r->m, r->v, r->L.count, lr_t, 0.9f, 0.999f, 1e-8f, r->step, r->W, s) !=
                hipSuccess) {
                rc = set_error(TM_EDEVICE, "adam");
                break;
            }
            if (h_loss && first == 0) {
                // loss of the first batch of the epoch, on the weights before the update
                hipLaunchKernelGGL(k_loss, dim3(64), dim3(256), 0, s, r->B.Y, r->B.T, rows, d_part);
                std::vector<double> lp(64);
                if (hipMemcpyAsync(lp.data(), d_part, 64 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    rc = set_error(TM_EDEVICE, "loss readback");
                    break;
                }
                for (double x : lp) loss_sum += x;
                loss_rows += rows;
            }
        }
        if (h_loss && loss_rows) h_loss[ep] = (float)(loss_sum / (double)(loss_rows * kOut));
    }
    (void)hipStreamSynchronize(s);
    if (d_part) (void)hipFree(d_part);
    if (d_T) (void)hipFree(d_T);
    if (d_perm) (void)hipFree(d_perm);
    return rc;
}

int tm_ranker_save(const tm_ranker* r, const char* path) {
    if (!r || !path) return set_error(TM_EINVAL, "null argument");
    std::vector<float> h((size_t)r->L.count * 3);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(h.data(), r->p, r->L.count * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.data() + r->L.count, r->m, r->L.count * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(h.data() + 2 * r->L.count, r->v, r->L.count * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(TM_EDEVICE, "read parameters");
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(TM_EINVAL, "cannot open %s", path);
    const char magic[8] = {'T', 'M', 'R', 'A', 'N', 'K', '0', '1'};
    const int64_t hdr[4] = {kFeat, kWidth, kOut, r->L.count};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 8, 4, f) == 4 &&
              std::fwrite(r->mu, 4, kOut, f) == (size_t)kOut && std::fwrite(r->sigma, 4, kOut, f) == (size_t)kOut &&
              std::fwrite(&r->step, 8, 1, f) == 1 && std::fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? TM_OK : set_error(TM_EINVAL, "write %s", path);
}

int tm_ranker_load(const char* path, tm_ranker** out) {
    if (!path || !out) return set_error(TM_EINVAL, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(TM_EINVAL, "cannot open %s", path);
    char magic[8];
    int64_t hdr[4];
    tm_ranker* r = nullptr;
    int rc = tm_ranker_create(0, &r);
    std::vector<float> h;
    if (rc == TM_OK) {
        const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TMRANK01", 8) == 0 &&
                        std::fread(hdr, 8, 4, f) == 4 && hdr[0] == kFeat && hdr[1] == kWidth && hdr[2] == kOut &&
                        hdr[3] == r->L.count && std::fread(r->mu, 4, kOut, f) == (size_t)kOut &&
                        std::fread(r->sigma, 4, kOut, f) == (size_t)kOut && std::fread(&r->step, 8, 1, f) == 1;
        if (ok) {
            h.resize((size_t)r->L.count * 3);
            if (std::fread(h.data(), 4, h.size(), f) != h.size()) rc = set_error(TM_EINVAL, "truncated %s", path);
        } else {
            rc = set_error(TM_EINVAL, "%s is not a ranker file of this layout", path);
        }
    }
    std::fclose(f);
    if (rc == TM_OK) {
        if (hipMemcpy(r->p, h.data(), r->L.count * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(r->m, h.data() + r->L.count, r->L.count * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(r->v, h.data() + 2 * r->L.count, r->L.count * 4, hipMemcpyHostToDevice) != hipSuccess ||
            launch_publish(r->p, r->L.count, r->W, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            rc = set_error(TM_EDEVICE, "upload parameters");
    }
    if (rc != TM_OK) {
        tm_ranker_destroy(r);
        return rc;
    }
    *out = r;
    return TM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ ranked search

namespace tmk {

int plan_ranked_search(tm_plan* p, tm_ranker* r, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk,
                       float lambda, float margin, int64_t* d_best, tm_stencil_cost* d_best_cost, hipStream_t s);

}  // namespace tmk

extern "C" int tm_ranker_features(const tm_plan* p, float* d_feat, void* stream) {
    return tmk::plan_features(p, d_feat, (hipStream_t)stream);
}

extern "C" int tm_ranker_block_estimates(const tm_plan* p, double* d_est, void* stream) {
    return tmk::plan_block_estimates(p, d_est, (hipStream_t)stream);
}

extern "C" int tm_search(tm_plan* p, tm_ranker* r, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk,
                         float lambda, float margin, int64_t* d_best, tm_stencil_cost* d_best_cost, void* stream) {
    if (!r) return tmk::plan_exhaustive_search(p, seg, nseg, d_best, d_best_cost, (hipStream_t)stream);
    if (!(margin >= 0.f)) return tmk::set_error(TM_EINVAL, "margin must be >= 0");
    return tmk::plan_ranked_search(p, r, seg, nseg, prefilter, topk, lambda, margin, d_best, d_best_cost,
                                   (hipStream_t)stream);
}

namespace tmk {

int plan_ranked_search(tm_plan* p, tm_ranker* r, const int64_t* seg, int64_t nseg, int32_t prefilter, int32_t topk,
                       float lambda, float margin, int64_t* d_best, tm_stencil_cost* d_best_cost, hipStream_t s) {
    if (!d_best) return set_error(TM_EINVAL, "null output");
    SearchBufs* sb = nullptr;
    int rc = plan_search_prepare(p, seg, nseg, prefilter, topk, true, &sb, s);
    if (rc != TM_OK) return rc;
    const int64_t n = plan_size(p);
    const int64_t nsel = nseg * topk;
    // the network's score of every candidate: descriptor features, forward, residuals
    // over the descriptor estimate
    hipError_t e = launch_features(plan_cands(p), n, plan_halo(p), chain_estimates(sb->cross, n), sb->X, nullptr, s);
    if (e == hipSuccess) e = launch_mlp_forward(sb->X, n, r->W, sb->Y, nullptr, nullptr, nullptr, s);
    if (e == hipSuccess) e = launch_combine(sb->Y, chain_estimates(sb->cross, n), n, r->mu, r->sigma, lambda, sb->score, s);
    if (prefilter > 0) {
        // the network keeps `prefilter` per instance; their block-model estimates (chain
        // statistics) choose the topk
        const int64_t m = nseg * (int64_t)prefilter;
        if (e == hipSuccess) e = launch_select(sb->score, sb->seg, nseg, 0, prefilter, 0.f, nullptr, sb->pre, s);
        if (e == hipSuccess) e = launch_chain_stats(plan_cands(p), sb->pre, m, plan_max_vol(p), plan_halo(p), sb->cross, s);
        if (e == hipSuccess)
            e = launch_combine(nullptr, chain_estimates(sb->cross, m), m, r->mu, r->sigma, lambda, sb->score, s);
        if (e == hipSuccess) e = launch_select(sb->score, sb->seg, nseg, prefilter, topk, margin, sb->pre, sb->sel, s);
    } else if (e == hipSuccess) {
        e = launch_select(sb->score, sb->seg, nseg, 0, topk, margin, nullptr, sb->sel, s);
    }
    // the survivors' exact costs (their cost rows serve the gather as scratch first:
    // 32 bytes per survivor, 16 used)
    static_assert(sizeof(tm_stencil_cost) >= 2 * sizeof(int64_t), "gather scratch");
    if (e == hipSuccess)
        e = launch_gather(plan_cands(p), sb->sel, nsel, topk, plan_cells_per_item(p), sb->sub, sb->map, sb->sub_seg,
                          sb->sub_hdr, plan_hdr(p), reinterpret_cast<int64_t*>(sb->sub_out), s);
    if (e == hipSuccess) e = plan_eval_sub(p, sb, s);
    if (e == hipSuccess) e = launch_select_segments(sb->sub_out, sb->sub_seg, nseg, sb->sub_best, s, sb->map);
    if (e == hipSuccess)
        e = launch_map_best(sb->sub_best, sb->sub_seg, sb->map, sb->sub_out, nseg, sb->seg, d_best, d_best_cost, s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "ranked search: %s", hipGetErrorString(e));
    return TM_OK;
}

}  // namespace tmk
