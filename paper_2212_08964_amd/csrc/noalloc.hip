// skgemm_run_noalloc: skgemm_run with the fix-up workspace in a device array
// the library owns, for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that must not call hipMalloc).
//
// The array `scratch` lives in the library's code object: every GPU the
// library runs on holds one copy (kScratchBytes) from module load until the
// process ends, zero-filled at load.  Its address differs per device and is
// obtained once per device with hipGetSymbolAddress; host code uses only that
// address, never the array's name (which on the host is a stand-in, not a
// device address).  Every call on a GPU shares that GPU's copy: calls that
// overlap in time on one GPU (two streams) race on it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "skgemm.h"
#include "skgemm_internal.h"

namespace {

// Header (error word), the fixed flag area, then the partial tiles:
// 64 MiB holds 254 FP32 partial tiles of 256 x 256 or 1020 of 128 x 128.
constexpr size_t kScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch`, looked up once per device.
skgemm_status_t scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SKGEMM_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SKGEMM_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SKGEMM_OK;
}

// Zero n int32 words from p (the error word and the flag lines a plan uses):
// a fill kernel rather than a memset, so that the call can be captured.
__global__ void __launch_bounds__(256) clear_words(int32_t* p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

}  // namespace

extern "C" skgemm_status_t skgemm_run_noalloc(skgemm_plan_t plan, const void* A, int64_t lda, const void* B,
                                              int64_t ldb, void* C, int64_t ldc, float alpha, float beta,
                                              const float* scale_a, const float* scale_b, hipStream_t stream) {
    // the fix-up part of the workspace only (plan_info field 28): the
    // operand re-layout a full-size workspace allows is not done here
    int64_t info[29] = {};
    skgemm_status_t st = skgemm_plan_info(plan, info, 29);
    if (st != SKGEMM_OK) return st;
    const size_t need = size_t(info[28]);
    if (need > kScratchBytes) return SKGEMM_ERR_WORKSPACE;
    if (need == 0) return skgemm_run(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, nullptr, 0, stream);
    void* ws = nullptr;
    st = scratch_ptr(&ws);
    if (st != SKGEMM_OK) return st;
    const int64_t g_sk = info[13];
    // The flags are left at zero by every run that completes its waits; an
    // earlier run whose wait timed out (or that overlapped this one) may have
    // left some raised, so the error word and this plan's flag lines are
    // cleared first, on the same stream.
    const int words = int((skg::kWsHeaderBytes + size_t(g_sk) * skg::kFlagStrideInts * 4) / 4);
    clear_words<<<(words + 255) / 256, 256, 0, stream>>>(reinterpret_cast<int32_t*>(ws), words);
    if (hipGetLastError() != hipSuccess) return SKGEMM_ERR_HIP;
    return skgemm_run(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, ws, need, stream);
}
