// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_f8(bool akc, bool bkc) {
    if (akc && bkc) return reinterpret_cast<const void*>(&skgemm_kernel<DT_F8, true, true>);
    return nullptr;
}

int kernel_threads_f8() { return kThreadsOf<DT_F8>; }

}  // namespace skg
