// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_bf16(bool akc, bool bkc) {
    if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_BF16, true, true>)
                        : reinterpret_cast<const void*>(&skgemm_kernel<DT_BF16, true, false>);
    return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_BF16, false, true>)
               : reinterpret_cast<const void*>(&skgemm_kernel<DT_BF16, false, false>);
}

int kernel_threads_bf16() { return kThreadsOf<DT_BF16>; }

}  // namespace skg
