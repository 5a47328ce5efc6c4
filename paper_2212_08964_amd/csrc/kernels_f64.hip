// Instantiations of the Stream-K GEMM kernel for one input type (one
// translation unit per type so they compile in parallel).
#include "skgemm_kernel.hpp"

namespace skg {

const void* kernel_fn_f64(bool akc, bool bkc, int v) {
    if (v == 0) {
        if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, true, true, 0>)
                            : reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, true, false, 0>);
        return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, false, true, 0>)
                   : reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, false, false, 0>);
    }
    if (v == 1) {
        if (akc) return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, true, true, 1>)
                            : reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, true, false, 1>);
        return bkc ? reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, false, true, 1>)
                   : reinterpret_cast<const void*>(&skgemm_kernel<DT_F64, false, false, 1>);
    }
    return nullptr;
}

int kernel_threads_f64(int v) { return v == 0 ? kThreadsOf<DT_F64, 0> : v == 1 ? kThreadsOf<DT_F64, 1> : 0; }

}  // namespace skg
