// Re-layout of a GEMM operand whose lines (rows of its contiguous dimension)
// start at addresses that are not 128-byte aligned: every 128-byte row
// segment of a k-slab then spans two cache lines and moves from L2 twice, so
// the plan may copy the operand into workspace lines of a 128-byte multiple
// before the GEMM (skgemm_run decides per call from the leading dimension).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "skgemm_internal.h"

namespace skg {

namespace {

constexpr int kPackThreads = 256;
constexpr int kPackBlocks = 2048;

// 16-byte chunks (line l, chunk c) in grid-stride order: consecutive threads
// take consecutive chunks of a line.  The destination chunk is 16-byte
// aligned (its lines are 128-byte multiples); the source chunk is read as one
// 16-byte load at the element alignment the caller's leading dimension gives
// (unaligned global loads are legal on this target).  A line's last partial
// chunk is copied element by element.
template <class T>
__global__ void __launch_bounds__(kPackThreads) pack_lines(const T* __restrict__ src, int64_t ld, int64_t lines,
                                                           int64_t cols, T* __restrict__ dst, int64_t ldd) {
    constexpr int E = 16 / int(sizeof(T));
    const int64_t chunks = (cols + E - 1) / E;
    const int64_t total = lines * chunks;
    for (int64_t idx = int64_t(blockIdx.x) * kPackThreads + threadIdx.x; idx < total;
         idx += int64_t(gridDim.x) * kPackThreads) {
        const int64_t l = idx / chunks, c = idx - l * chunks;
        const T* s = src + l * ld + c * E;
        T* d = dst + l * ldd + c * E;
        if ((c + 1) * E <= cols) {
            uint4 v;
            __builtin_memcpy(&v, s, 16);
            *reinterpret_cast<uint4*>(d) = v;
        } else {
            for (int64_t e = 0; e < cols - c * E; ++e) d[e] = s[e];
        }
    }
}

}  // namespace

int launch_pack(const void* src, int64_t ld, int64_t lines, int64_t cols, void* dst, int64_t ldd, int eb,
                void* stream) {
    if (lines <= 0 || cols <= 0) return int(hipSuccess);
    const int64_t chunks = lines * ((cols * eb + 15) / 16);
    const int64_t blocks = std::min<int64_t>(kPackBlocks, (chunks + kPackThreads - 1) / kPackThreads);
    const dim3 grid{unsigned(blocks)}, block{unsigned(kPackThreads)};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (eb) {
        case 1:
            pack_lines<uint8_t><<<grid, block, 0, s>>>(static_cast<const uint8_t*>(src), ld, lines, cols,
                                                      static_cast<uint8_t*>(dst), ldd);
            break;
        case 2:
            pack_lines<uint16_t><<<grid, block, 0, s>>>(static_cast<const uint16_t*>(src), ld, lines, cols,
                                                       static_cast<uint16_t*>(dst), ldd);
            break;
        case 4:
            pack_lines<uint32_t><<<grid, block, 0, s>>>(static_cast<const uint32_t*>(src), ld, lines, cols,
                                                       static_cast<uint32_t*>(dst), ldd);
            break;
        case 8:
            pack_lines<uint64_t><<<grid, block, 0, s>>>(static_cast<const uint64_t*>(src), ld, lines, cols,
                                                       static_cast<uint64_t*>(dst), ldd);
            break;
        default:
            return int(hipErrorInvalidValue);
    }
    return int(hipGetLastError());
}

}  // namespace skg
