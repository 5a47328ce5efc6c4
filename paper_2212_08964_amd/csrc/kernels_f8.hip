// Lean instantiations (plain GEMMs) of the Stream-K GEMM kernel for one
// input type, and its workgroup sizes.
#include "kernel_tables.hpp"

namespace skg {

const void* kernel_fn_f8(bool akc, bool bkc, int v) { return kernel_table<DT_F8, false>(akc, bkc, v); }

int kernel_threads_f8(int v) { return v == 0 ? kThreadsOf<DT_F8, 0> : v == 1 ? kThreadsOf<DT_F8, 1> : 0; }

}  // namespace skg
