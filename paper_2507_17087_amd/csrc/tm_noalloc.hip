// tm_noalloc.hip -- tm_eval_stencil_batch_noalloc: the stencil evaluation of
// tm_eval_stencil_batch for callers that cannot allocate device memory.  Its batch
// header, descriptors, table arena and work counter live in `scratch`, a file-scope
// device array of TM_NOALLOC_SCRATCH_BYTES held by every GPU the library runs on
// until the process ends.  Host code never uses the array's name as an address (it
// is a host-side stand-in): the device address comes from hipGetSymbolAddress, once
// per device, and only that pointer is passed to the kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tm_internal.h"
#include "tm_plan.h"

namespace tmk {

static __device__ __align__(256) unsigned char scratch[TM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::once_flag g_once[kMaxDevices];
static void* g_ptr[kMaxDevices];
static hipError_t g_err[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up on the first call
// on each device, with that device current).
static int scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(TM_ENOTSUP, "device %d", dev);
    std::call_once(g_once[dev], [dev]() {
        void* p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
    });
    if (g_err[dev] != hipSuccess || !g_ptr[dev])
        return set_error(TM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(g_err[dev]));
    *out = g_ptr[dev];
    return TM_OK;
}

static int64_t up256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace tmk

using namespace tmk;

extern "C" int tm_eval_stencil_batch_noalloc(const tm_candidate* c, int64_t n, const tm_stencil* st,
                                             tm_stencil_cost* d_out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (!st) return set_error(TM_EINVAL, "null stencil");
    Compiled cp;
    int rc = compile_batch(c, n, st, 0, true, cp);
    if (rc != TM_OK) return rc;
    if (n == 0) return TM_OK;
    if (!d_out) return set_error(TM_EINVAL, "null output");
    // scratch layout: header | descriptors | table arena | work counter
    const int64_t o_cands = up256((int64_t)sizeof(DevHeader));
    const int64_t o_arena = o_cands + up256(n * (int64_t)sizeof(DevCand));
    const int64_t o_count = o_arena + up256(cp.arena_words * 4);
    const int64_t need = o_count + 256;
    if (need > (int64_t)TM_NOALLOC_SCRATCH_BYTES)
        return set_error(TM_ECAPACITY, "the batch needs %lld bytes of scratch; the library holds %lld",
                         (long long)need, (long long)TM_NOALLOC_SCRATCH_BYTES);
    char* base = nullptr;
    rc = scratch_ptr((void**)&base);
    if (rc != TM_OK) return rc;
    DevHeader* hdr = reinterpret_cast<DevHeader*>(base);
    DevCand* cands = reinterpret_cast<DevCand*>(base + o_cands);
    int32_t* arena = reinterpret_cast<int32_t*>(base + o_arena);
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(base + o_count);
    // the descriptors go up from this call's host memory; waiting for the copies keeps
    // it alive until they are done (nothing here allocates pinned staging)
    hipError_t e = hipMemcpyAsync(hdr, &cp.hdr, sizeof(DevHeader), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cands, cp.cands.data(), (size_t)n * sizeof(DevCand), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // the table build writes the whole arena (tables and item table) and zeroes the
    // outputs and both counters before the counting starts
    const bool fin = n <= kFinInCount;
    if (e == hipSuccess) e = launch_build_tables(hdr, cands, n, arena, 1, s, d_out, counter);
    if (e == hipSuccess)
        e = launch_count(hdr, cands, arena, counter, d_out, count_grid(cp.cnt_words, cp.items, 0), cp.cnt_words, s,
                         fin, nullptr);
    if (e == hipSuccess && !fin) e = launch_finalize_select(hdr, d_out, nullptr, n, s);
    if (e != hipSuccess) return set_error(TM_EDEVICE, "stencil launch (no allocation): %s", hipGetErrorString(e));
    return TM_OK;
}
