// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_f8(bool akc, bool bkc, int v) {
    if (!akc || !bkc) return nullptr;
    if (v == 0) return reinterpret_cast<const void*>(&skgemm_kernel<DT_F8, true, true, 0>);
    if (v == 1) return reinterpret_cast<const void*>(&skgemm_kernel<DT_F8, true, true, 1>);
    return nullptr;
}

int kernel_threads_f8(int v) { return v == 0 ? kThreadsOf<DT_F8, 0> : v == 1 ? kThreadsOf<DT_F8, 1> : 0; }

}  // namespace skg
