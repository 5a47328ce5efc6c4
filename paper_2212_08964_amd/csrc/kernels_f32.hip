// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_f32(bool akc, bool bkc) {
    if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F32, true, true>)
                        : reinterpret_cast<const void*>(&skgemm_kernel<DT_F32, true, false>);
    return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F32, false, true>)
               : reinterpret_cast<const void*>(&skgemm_kernel<DT_F32, false, false>);
}

int kernel_threads_f32() { return kThreadsOf<DT_F32>; }

}  // namespace skg
