// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_f16(bool akc, bool bkc, int v) {
    if (v == 0) {
        if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, true, 0>)
                            : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, false, 0>);
        return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, true, 0>)
                   : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, false, 0>);
    }
    if (v == 1) {
        if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, true, 1>)
                            : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, false, 1>);
        return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, true, 1>)
                   : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, false, 1>);
    }
    if (v == 2) {
        if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, true, 2>)
                            : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, false, 2>);
        return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, true, 2>)
                   : reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, false, false, 2>);
    }
    // implicit-GEMM convolution: A gathered, filters K-contiguous
    if (v == 3 && akc && bkc) return reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, true, 3>);
    if (v == 4 && akc && bkc) return reinterpret_cast<const void*>(&skgemm_kernel<DT_F16, true, true, 4>);
    return nullptr;
}

int kernel_threads_f16(int v) {
    return v == 0 ? kThreadsOf<DT_F16, 0> : v == 1 ? kThreadsOf<DT_F16, 1> : v == 2 ? kThreadsOf<DT_F16, 2>
           : v == 3 ? kThreadsOf<DT_F16, 3> : v == 4 ? kThreadsOf<DT_F16, 4> : 0;
}

}  // namespace skg
