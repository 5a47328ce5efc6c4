// Full instantiations (group table, batch, trace, timestamps) of the
// Stream-K GEMM kernel for one input type.
#include "kernel_tables.hpp"

namespace skg {

const void* kernel_fn_f32_full(bool akc, bool bkc, int v) { return kernel_table<DT_F32, true>(akc, bkc, v); }

}  // namespace skg
