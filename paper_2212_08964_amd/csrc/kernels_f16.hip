// Lean instantiations (plain GEMMs) of the Stream-K GEMM kernel for one
// input type, and its workgroup sizes.
#include "kernel_tables.hpp"

namespace skg {

const void* kernel_fn_f16(bool akc, bool bkc, int v) { return kernel_table<DT_F16, false>(akc, bkc, v); }

int kernel_threads_f16(int v) { return v == 0 ? kThreadsOf<DT_F16, 0> : v == 1 ? kThreadsOf<DT_F16, 1> : v == 2 ? kThreadsOf<DT_F16, 2> : v == 3 ? kThreadsOf<DT_F16, 3> : v == 4 ? kThreadsOf<DT_F16, 4> : v == 5 ? kThreadsOf<DT_F16, 5> : v == 6 ? kThreadsOf<DT_F16, 6> : v == 7 ? kThreadsOf<DT_F16, 7> : v == 8 ? kThreadsOf<DT_F16, 8> : v == 9 ? kThreadsOf<DT_F16, 9> : 0; }

}  // namespace skg
