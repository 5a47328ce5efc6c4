// Kernel tables: the instantiations of the Stream-K GEMM kernel that exist
// for each input type, tile variant and operand contiguity, in their lean
// (plain GEMM) or full (group table, batch, trace, timestamps) form.  Each
// translation unit instantiates one (type, form) table, so they compile in
// parallel.
#pragma once

#include "skgemm_kernel.hpp"

namespace skg {

template <int DT, bool AKC, bool BKC, int V, bool FULL>
const void* kernel_ptr() {
    return reinterpret_cast<const void*>(&skgemm_kernel<DT, AKC, BKC, V, FULL>);
}

// every combination of operand contiguity
template <int DT, int V, bool FULL>
const void* any_layout(bool akc, bool bkc) {
    if (akc) return bkc ? kernel_ptr<DT, true, true, V, FULL>() : kernel_ptr<DT, true, false, V, FULL>();
    return bkc ? kernel_ptr<DT, false, true, V, FULL>() : kernel_ptr<DT, false, false, V, FULL>();
}

// K-contiguous A, either B (the skinny tile: a 64-row MN-contiguous slab has
// rows shorter than the slab layout's minimum)
template <int DT, int V, bool FULL>
const void* akc_only(bool akc, bool bkc) {
    if (!akc) return nullptr;
    return bkc ? kernel_ptr<DT, true, true, V, FULL>() : kernel_ptr<DT, true, false, V, FULL>();
}

// either A, K-contiguous B (the tall tile: a 64-column MN-contiguous slab has
// rows shorter than the slab layout's minimum)
template <int DT, int V, bool FULL>
const void* bkc_only(bool akc, bool bkc) {
    if (!bkc) return nullptr;
    return akc ? kernel_ptr<DT, true, true, V, FULL>() : kernel_ptr<DT, false, true, V, FULL>();
}

// K-contiguous A and B only (FP8; the convolution kernels)
template <int DT, int V, bool FULL>
const void* kc_only(bool akc, bool bkc) {
    return akc && bkc ? kernel_ptr<DT, true, true, V, FULL>() : nullptr;
}

template <int DT, bool FULL>
const void* kernel_table(bool akc, bool bkc, int v) {
    if constexpr (DT == DT_BF16 || DT == DT_F16) {
        switch (v) {
            case 0: return any_layout<DT, 0, FULL>(akc, bkc);
            case 1: return any_layout<DT, 1, FULL>(akc, bkc);
            case 2: return any_layout<DT, 2, FULL>(akc, bkc);
            case 3: return kc_only<DT, 3, FULL>(akc, bkc);    // implicit-GEMM convolution
            case 4: return kc_only<DT, 4, FULL>(akc, bkc);
            case 5: return akc_only<DT, 5, FULL>(akc, bkc);    // skinny tile
            case 6: return bkc_only<DT, 6, FULL>(akc, bkc);    // tall tile
            case 7: return kc_only<DT, 7, FULL>(akc, bkc);     // tall tile, convolution
            case 8: return any_layout<DT, 8, FULL>(akc, bkc);  // small tile, three stages
            case 9: return kc_only<DT, 9, FULL>(akc, bkc);     // the same, convolution
            default: return nullptr;
        }
    } else if constexpr (DT == DT_F8) {
        switch (v) {
            case 0: return kc_only<DT, 0, FULL>(akc, bkc);
            case 1: return kc_only<DT, 1, FULL>(akc, bkc);
            default: return nullptr;
        }
    } else if constexpr (DT == DT_F64) {
        switch (v) {
            case 0: return any_layout<DT, 0, FULL>(akc, bkc);
            case 1: return any_layout<DT, 1, FULL>(akc, bkc);
            default: return nullptr;
        }
    } else {
        static_assert(DT == DT_F32, "input types");
        return v == 0 ? any_layout<DT, 0, FULL>(akc, bkc) : nullptr;
    }
}

}  // namespace skg
