// Kernel lookup, occupancy query and launch for the Stream-K GEMM kernels.
#include <hip/hip_runtime.h>

#include "skgemm_internal.h"

namespace skg {

const void* kernel_fn_f32(bool akc, bool bkc, int v);
const void* kernel_fn_f16(bool akc, bool bkc, int v);
const void* kernel_fn_bf16(bool akc, bool bkc, int v);
const void* kernel_fn_f8(bool akc, bool bkc, int v);
const void* kernel_fn_f64(bool akc, bool bkc, int v);
const void* kernel_fn_f32_full(bool akc, bool bkc, int v);
const void* kernel_fn_f16_full(bool akc, bool bkc, int v);
const void* kernel_fn_bf16_full(bool akc, bool bkc, int v);
const void* kernel_fn_f8_full(bool akc, bool bkc, int v);
const void* kernel_fn_f64_full(bool akc, bool bkc, int v);
int kernel_threads_f32(int v);
int kernel_threads_f16(int v);
int kernel_threads_bf16(int v);
int kernel_threads_f8(int v);
int kernel_threads_f64(int v);

// full: the instantiation with the group table, batch, trace and timestamp
// paths (every lean kernel has one)
static const void* kernel_for(int dtype, bool akc, bool bkc, int v, bool full) {
    switch (dtype) {
        case DT_F32: return full ? kernel_fn_f32_full(akc, bkc, v) : kernel_fn_f32(akc, bkc, v);
        case DT_F16: return full ? kernel_fn_f16_full(akc, bkc, v) : kernel_fn_f16(akc, bkc, v);
        case DT_BF16: return full ? kernel_fn_bf16_full(akc, bkc, v) : kernel_fn_bf16(akc, bkc, v);
        case DT_F8: return full ? kernel_fn_f8_full(akc, bkc, v) : kernel_fn_f8(akc, bkc, v);
        case DT_F64: return full ? kernel_fn_f64_full(akc, bkc, v) : kernel_fn_f64(akc, bkc, v);
        default: return nullptr;
    }
}

static bool needs_full(const KArgs& a) { return a.G || a.batch > 1 || a.trace || a.times; }

bool kernel_exists(int dtype, bool akc, bool bkc, int v) {
    return kernel_for(dtype, akc, bkc, v, false) != nullptr && kernel_for(dtype, akc, bkc, v, true) != nullptr;
}

int kernel_threads(int dtype, int v) {
    switch (dtype) {
        case DT_F32: return kernel_threads_f32(v);
        case DT_F16: return kernel_threads_f16(v);
        case DT_BF16: return kernel_threads_bf16(v);
        case DT_F8: return kernel_threads_f8(v);
        case DT_F64: return kernel_threads_f64(v);
        default: return 0;
    }
}

// The smaller of the two forms' occupancies: a plan's grid must be co-resident
// whichever form runs it.
int kernel_occupancy(int dtype, bool akc, bool bkc, int v) {
    int occ = 0;
    for (const bool full : {false, true}) {
        const void* f = kernel_for(dtype, akc, bkc, v, full);
        if (!f) return 0;
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kernel_threads(dtype, v), 0) != hipSuccess) return 0;
        occ = full ? (n < occ ? n : occ) : n;
    }
    return occ;
}

int launch_gemm(int dtype, bool akc, bool bkc, int v, const KArgs& args, int grid, void* stream) {
    const void* f = kernel_for(dtype, akc, bkc, v, needs_full(args));
    if (!f) return int(hipErrorInvalidDeviceFunction);
    KArgs copy = args;
    void* params[] = {&copy};
    return int(hipLaunchKernel(f, dim3(grid), dim3(kernel_threads(dtype, v)), params, 0,
                               reinterpret_cast<hipStream_t>(stream)));
}

}  // namespace skg
