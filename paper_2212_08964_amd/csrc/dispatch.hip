// Kernel lookup, occupancy query and launch for the Stream-K GEMM kernels.
#include <hip/hip_runtime.h>

#include "skgemm_internal.h"

namespace skg {

const void* kernel_fn_f32(bool akc, bool bkc);
const void* kernel_fn_f16(bool akc, bool bkc);
const void* kernel_fn_bf16(bool akc, bool bkc);
const void* kernel_fn_f8(bool akc, bool bkc);
int kernel_threads_f32();
int kernel_threads_f16();
int kernel_threads_bf16();
int kernel_threads_f8();

static const void* kernel_for(int dtype, bool akc, bool bkc) {
    switch (dtype) {
        case DT_F32: return kernel_fn_f32(akc, bkc);
        case DT_F16: return kernel_fn_f16(akc, bkc);
        case DT_BF16: return kernel_fn_bf16(akc, bkc);
        case DT_F8: return kernel_fn_f8(akc, bkc);
        default: return nullptr;
    }
}

bool kernel_exists(int dtype, bool akc, bool bkc) { return kernel_for(dtype, akc, bkc) != nullptr; }

int kernel_threads(int dtype) {
    switch (dtype) {
        case DT_F32: return kernel_threads_f32();
        case DT_F16: return kernel_threads_f16();
        case DT_BF16: return kernel_threads_bf16();
        case DT_F8: return kernel_threads_f8();
        default: return 0;
    }
}

int kernel_occupancy(int dtype, bool akc, bool bkc) {
    const void* f = kernel_for(dtype, akc, bkc);
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kernel_threads(dtype), 0) != hipSuccess) return 0;
    return n;
}

int launch_gemm(int dtype, bool akc, bool bkc, const KArgs& args, int grid, void* stream) {
    const void* f = kernel_for(dtype, akc, bkc);
    if (!f) return int(hipErrorInvalidDeviceFunction);
    KArgs copy = args;
    void* params[] = {&copy};
    return int(hipLaunchKernel(f, dim3(grid), dim3(kernel_threads(dtype)), params, 0,
                               reinterpret_cast<hipStream_t>(stream)));
}

}  // namespace skg
