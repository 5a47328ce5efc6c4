// Lean instantiations (plain GEMMs) of the Stream-K GEMM kernel for one
// input type, and its workgroup sizes.
#include "kernel_tables.hpp"

namespace skg {

const void* kernel_fn_bf16(bool akc, bool bkc, int v) { return kernel_table<DT_BF16, false>(akc, bkc, v); }

int kernel_threads_bf16(int v) { return v == 0 ? kThreadsOf<DT_BF16, 0> : v == 1 ? kThreadsOf<DT_BF16, 1> : v == 2 ? kThreadsOf<DT_BF16, 2> : v == 3 ? kThreadsOf<DT_BF16, 3> : v == 4 ? kThreadsOf<DT_BF16, 4> : v == 5 ? kThreadsOf<DT_BF16, 5> : v == 6 ? kThreadsOf<DT_BF16, 6> : v == 7 ? kThreadsOf<DT_BF16, 7> : v == 8 ? kThreadsOf<DT_BF16, 8> : v == 9 ? kThreadsOf<DT_BF16, 9> : 0; }

}  // namespace skg
