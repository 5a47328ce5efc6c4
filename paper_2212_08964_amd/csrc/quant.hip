// Per-tensor FP8 (OCP E4M3FN) quantisation for the FP8 GEMM front end.
//
//   s = absmax(X) / 448   (1 when X is all zero), rounded to FP32
//   Q = E4M3_RNE(clamp(X / s, -448, 448))
//
// Two or three launches, all HBM-bound: absmax_partial reads X once (16-byte
// loads when rows are aligned) and writes one maximum per workgroup; the
// quantising kernel reduces those maxima to s in every workgroup (its first
// workgroup stores s for the GEMM), reads X again and writes the codes.  On
// grids of more than kFoldMaxBlocks workgroups a one-workgroup kernel
// (absmax_finish) reduces the maxima once instead, before the quantising
// kernel.  Nothing goes through the host and no memory needs clearing, so
// the sequence can be captured in a graph.  An empty X takes absmax_finish
// alone (s = 1).
// Where every row is 16-byte aligned the second kernel is quantize_rows
// (same storage order: 16 elements per thread, 16-byte loads and stores) or
// quantize_transpose (the FP8 GEMM wants both operands K-contiguous, so a
// row-major B changes order on the way out: 64x64 tiles through LDS, 16-byte
// loads and stores); otherwise quantize_tiles (element loads, 4-byte stores,
// any alignment).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "skgemm_internal.h"

namespace skg {

constexpr int kQThreads = 256;
constexpr int kAbsmaxBlocks = 1024;
constexpr float kE4M3Max = 448.0f;
constexpr int64_t kFoldMaxBlocks = 4096;   // quantising grids that reduce the maxima themselves

template <int DT>
__device__ __forceinline__ float elem(const void* x, int64_t i) {
    if constexpr (DT == DT_F32) return reinterpret_cast<const float*>(x)[i];
    else if constexpr (DT == DT_BF16) return __builtin_bit_cast(float, uint32_t(reinterpret_cast<const uint16_t*>(x)[i]) << 16);
    else return float(reinterpret_cast<const _Float16*>(x)[i]);
}

// |v| for finite v, 0 for NaN and infinities: the scale is taken over the
// finite entries (a non-finite entry is encoded as NaN, see to_e4m3x2).
__device__ __forceinline__ float fin_abs(float v) {
    const float a = fabsf(v);
    return a <= 3.40282347e38f ? a : 0.0f;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float block_max(float v, float* red) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (w == 0) {
        v = lane < int(blockDim.x >> 6) ? red[lane] : 0.0f;
        v = wave_max(v);
    }
    return v;
}

// Logical matrix `outer` x `inner` with the inner dimension contiguous and
// leading dimension ld; vec says 16-byte loads are aligned for every row.
template <int DT>
__global__ void __launch_bounds__(kQThreads) absmax_partial(const void* x, int64_t outer, int64_t inner, int64_t ld,
                                                            int vec, float* partial) {
    __shared__ float red[kQThreads / 64];
    constexpr int EB = DT == DT_F32 ? 4 : 2, VE = 16 / EB;
    float m = 0.0f;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    if (vec) {
        const int64_t vin = inner / VE;
        const int64_t n = outer * vin;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
            const int64_t o = i / vin, c = (i % vin) * VE;
            const uint4 u = *reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(x) + (o * ld + c) * EB);
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (DT == DT_F32) {
                    m = fmaxf(m, fin_abs(__builtin_bit_cast(float, w[e])));
                } else if constexpr (DT == DT_BF16) {
                    m = fmaxf(m, fin_abs(__builtin_bit_cast(float, w[e] << 16)));
                    m = fmaxf(m, fin_abs(__builtin_bit_cast(float, w[e] & 0xffff0000u)));
                } else {
                    m = fmaxf(m, fin_abs(float(__builtin_bit_cast(_Float16, uint16_t(w[e])))));
                    m = fmaxf(m, fin_abs(float(__builtin_bit_cast(_Float16, uint16_t(w[e] >> 16)))));
                }
            }
        }
    } else {
        const int64_t n = outer * inner;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
            const int64_t o = i / inner, c = i % inner;
            m = fmaxf(m, fin_abs(elem<DT>(x, o * ld + c)));
        }
    }
    m = block_max(m, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ void __launch_bounds__(kQThreads) absmax_finish(const float* partial, int n, float* scale) {
    __shared__ float red[kQThreads / 64];
    float m = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmaxf(m, partial[i]);
    m = block_max(m, red);
    if (threadIdx.x == 0) scale[0] = m == 0.0f ? 1.0f : m / kE4M3Max;
}

// s from the per-workgroup maxima of absmax_partial, computed by every
// workgroup of the quantising pass (the same formula as absmax_finish, so the
// same bits); the first workgroup also stores it for the GEMM's epilogue.
// n = 0: absmax_finish has stored s already (large grids, where every
// workgroup reading all maxima would cost more than the extra launch).
// Every thread of the workgroup must call it.
__device__ __forceinline__ float scale_of(const float* partial, int n, float* scale, bool store) {
    if (n == 0) return *scale;
    __shared__ float red[kQThreads / 64];
    float m = 0.0f;
    for (int i = threadIdx.x; i < n; i += kQThreads) m = fmaxf(m, partial[i]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = red[0];
#pragma unroll
    for (int k = 1; k < kQThreads / 64; ++k) m = fmaxf(m, red[k]);
    const float s = m == 0.0f ? 1.0f : m / kE4M3Max;
    if (store && threadIdx.x == 0) scale[0] = s;
    return s;
}

// X / s rounded to FP32, clamped to the E4M3 range, rounded to E4M3 (nearest
// even) by the hardware conversion; two codes per call.
// A NaN or infinite input (E4M3FN has no infinity) becomes the NaN code
// 0x7f with the input's sign, so it reaches the product as NaN rather than
// as a clamped finite value.
template <bool HI>
__device__ __forceinline__ uint32_t to_e4m3x2(float a, float b, float s, uint32_t old) {
    const float qa = fminf(fmaxf(a / s, -kE4M3Max), kE4M3Max);
    const float qb = fminf(fmaxf(b / s, -kE4M3Max), kE4M3Max);
    uint32_t r = uint32_t(__builtin_amdgcn_cvt_pk_fp8_f32(qa, qb, int(old), HI));
    constexpr int SA = HI ? 16 : 0, SB = SA + 8;
    const uint32_t ua = __builtin_bit_cast(uint32_t, a), ub = __builtin_bit_cast(uint32_t, b);
    if ((ua & 0x7f800000u) == 0x7f800000u) r = (r & ~(0xffu << SA)) | ((0x7fu | ((ua >> 24) & 0x80u)) << SA);
    if ((ub & 0x7f800000u) == 0x7f800000u) r = (r & ~(0xffu << SB)) | ((0x7fu | ((ub >> 24) & 0x80u)) << SB);
    return r;
}

// One 64 x 64 tile of the logical rows x cols matrix per workgroup.  x_col /
// q_col select column-major storage of the input / output.
template <int DT>
__global__ void __launch_bounds__(kQThreads) quantize_tiles(const void* x, int64_t rows, int64_t cols, int64_t ldx,
                                                            int x_col, uint8_t* q, int64_t ldq, int q_col,
                                                            const float* partial, int np, float* scale) {
    __shared__ float tile[64][65];
    const float s = scale_of(partial, np, scale, blockIdx.x == 0 && blockIdx.y == 0);
    const int64_t r0 = int64_t(blockIdx.y) * 64, c0 = int64_t(blockIdx.x) * 64;
    const int t = threadIdx.x;
    // read: consecutive threads walk the input's contiguous dimension
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int idx = t + k * kQThreads;
        const int a = idx & 63, b = idx >> 6;      // a: contiguous index, b: strided index
        const int rl = x_col ? a : b, cl = x_col ? b : a;
        const int64_t r = r0 + rl, c = c0 + cl;
        float v = 0.0f;
        if (r < rows && c < cols) v = elem<DT>(x, x_col ? c * ldx + r : r * ldx + c);
        tile[rl][cl] = v;
    }
    __syncthreads();
    // write: each thread converts four consecutive elements of the output's
    // contiguous dimension
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int idx = t + k * kQThreads;           // 1024 groups of four
        const int a4 = (idx & 15) * 4, b = idx >> 4;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = q_col ? tile[a4 + e][b] : tile[b][a4 + e];
        const int64_t outer = (q_col ? c0 : r0) + b;
        const int64_t in0 = (q_col ? r0 : c0) + a4;
        const int64_t n_outer = q_col ? cols : rows, n_inner = q_col ? rows : cols;
        if (outer >= n_outer || in0 >= n_inner) continue;
        uint32_t w = to_e4m3x2<false>(v[0], v[1], s, 0u);
        w = to_e4m3x2<true>(v[2], v[3], s, w);
        uint8_t* dst = q + outer * ldq + in0;
        if (in0 + 4 <= n_inner && (reinterpret_cast<uintptr_t>(dst) & 3) == 0) {
            *reinterpret_cast<uint32_t*>(dst) = w;
        } else {
            for (int e = 0; e < 4 && in0 + e < n_inner; ++e) dst[e] = uint8_t(w >> (8 * e));
        }
    }
}

// Eight codes of two 16-byte input words of a 16-bit type, or four of one
// FP32 word: the input vector's elements in order.
template <int DT>
__device__ __forceinline__ void unpack(const uint4& u, float* v) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if constexpr (DT == DT_F32) {
            v[e] = __builtin_bit_cast(float, w[e]);
        } else if constexpr (DT == DT_BF16) {
            v[2 * e] = __builtin_bit_cast(float, w[e] << 16);
            v[2 * e + 1] = __builtin_bit_cast(float, w[e] & 0xffff0000u);
        } else {
            v[2 * e] = float(__builtin_bit_cast(_Float16, uint16_t(w[e])));
            v[2 * e + 1] = float(__builtin_bit_cast(_Float16, uint16_t(w[e] >> 16)));
        }
    }
}

// Sixteen codes of v[0..15] as one 16-byte word.
__device__ __forceinline__ uint4 codes16(const float* v, float s) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w[i] = to_e4m3x2<false>(v[4 * i], v[4 * i + 1], s, 0u);
        w[i] = to_e4m3x2<true>(v[4 * i + 2], v[4 * i + 3], s, w[i]);
    }
    return uint4{w[0], w[1], w[2], w[3]};
}

// Same storage order in and out (`outer` rows of `inner` contiguous
// elements), inner a multiple of 16 and every row 16-byte aligned on both
// sides: each thread converts 16 consecutive elements of one row with 16-byte
// loads and one 16-byte store.
template <int DT>
__global__ void __launch_bounds__(kQThreads) quantize_rows(const void* x, int64_t groups, int64_t per_row, int64_t ldx,
                                                           uint8_t* q, int64_t ldq, const float* partial, int np,
                                                           float* scale) {
    constexpr int EB = DT == DT_F32 ? 4 : 2, NV = 16 * EB / 16;   // input vectors per group
    const float s = scale_of(partial, np, scale, blockIdx.x == 0);
    const int64_t g = int64_t(blockIdx.x) * kQThreads + threadIdx.x;
    if (g >= groups) return;
    const int64_t o = g / per_row, c = (g - o * per_row) * 16;
    const uint4* src = reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(x) + (o * ldx + c) * EB);
    uint4 u[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) u[k] = src[k];
    float v[16];
#pragma unroll
    for (int k = 0; k < NV; ++k) unpack<DT>(u[k], v + k * (16 / NV));
    *reinterpret_cast<uint4*>(q + o * ldq + c) = codes16(v, s);
}

// Transposing form: X stored as `outer` rows of `inner` contiguous elements,
// Q stored as `inner` rows of `outer` contiguous codes.  One 64 x 64 tile per
// workgroup through LDS: 16-byte loads along X's rows, 16-byte stores along
// Q's.  Needs inner a multiple of the elements per 16 bytes, outer a multiple
// of 16 and 16-byte aligned rows on both sides.
template <int DT>
__global__ void __launch_bounds__(kQThreads) quantize_transpose(const void* x, int64_t outer, int64_t inner,
                                                                int64_t ldx, uint8_t* q, int64_t ldq,
                                                                const float* partial, int np, float* scale) {
    constexpr int EB = DT == DT_F32 ? 4 : 2, VE = 16 / EB, VPR = 64 / VE, LOADS = 64 * VPR / kQThreads;
    __shared__ float tile[64][65];
    const float s = scale_of(partial, np, scale, blockIdx.x == 0 && blockIdx.y == 0);
    const int64_t i0 = int64_t(blockIdx.x) * 64, o0 = int64_t(blockIdx.y) * 64;
    const int t = threadIdx.x;
    uint4 u[LOADS];
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int idx = t + k * kQThreads, row = idx / VPR, vc = idx % VPR;
        const int64_t o = o0 + row, i = i0 + int64_t(vc) * VE;
        u[k] = uint4{0u, 0u, 0u, 0u};
        if (o < outer && i < inner)
            u[k] = *reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(x) + (o * ldx + i) * EB);
    }
#pragma unroll
    for (int k = 0; k < LOADS; ++k) {
        const int idx = t + k * kQThreads, row = idx / VPR, vc = idx % VPR;
        float v[VE];
        unpack<DT>(u[k], v);
#pragma unroll
        for (int e = 0; e < VE; ++e) tile[row][vc * VE + e] = v[e];
    }
    __syncthreads();
    // Q row (X column) and group of 16 X rows: four neighbouring lanes write
    // the 64 contiguous codes of one Q row
    const int ic = t >> 2, rg = t & 3;
    const int64_t i = i0 + ic, o = o0 + 16 * rg;
    if (i >= inner || o >= outer) return;
    float v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = tile[16 * rg + e][ic];
    *reinterpret_cast<uint4*>(q + i * ldq + o) = codes16(v, s);
}

int quant_workspace_floats() { return kAbsmaxBlocks; }

int launch_quantize(int dtype, const void* x, int64_t rows, int64_t cols, int64_t ldx, bool x_col, uint8_t* q,
                    int64_t ldq, bool q_col, float* scale, float* partial, void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t outer = x_col ? cols : rows, inner = x_col ? rows : cols;
    const int eb = dtype == DT_F32 ? 4 : 2;
    const bool vec = (inner * eb) % 16 == 0 && (ldx * eb) % 16 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    const int64_t work = vec ? outer * (inner / (16 / eb)) : outer * inner;
    const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(kAbsmaxBlocks, (work + kQThreads - 1) / kQThreads)));
    const dim3 tiles(unsigned((cols + 63) / 64), unsigned((rows + 63) / 64));
    const bool any = rows > 0 && cols > 0;
    // vectorised forms where every row is 16-byte aligned on both sides
    const auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool rows_ok = (ldx * eb) % 16 == 0 && a16(x) && ldq % 16 == 0 && a16(q);
    const int form = !any || !rows_ok ? 0
                     : x_col == q_col ? (inner % 16 == 0 ? 1 : 0)
                                      : (inner % (16 / eb) == 0 && outer % 16 == 0 ? 2 : 0);
    const int64_t groups = outer * (inner / 16);
    const unsigned row_blocks = unsigned((groups + kQThreads - 1) / kQThreads);
    const dim3 ttiles(unsigned((inner + 63) / 64), unsigned((outer + 63) / 64));
    // the quantising pass reduces the maxima itself when its grid is small
    // (one launch fewer); larger grids keep the one-workgroup reduction
    const int64_t qblocks = form == 1 ? int64_t(row_blocks)
                            : form == 2 ? int64_t(ttiles.x) * ttiles.y : int64_t(tiles.x) * tiles.y;
    const int np = any && qblocks <= kFoldMaxBlocks ? blocks : 0;
#define SKG_QUANT(DT_)                                                                                         \
    absmax_partial<DT_><<<blocks, kQThreads, 0, st>>>(x, outer, inner, ldx, vec, partial);                     \
    if (np == 0) absmax_finish<<<1, kQThreads, 0, st>>>(partial, blocks, scale);                               \
    if (form == 1)                                                                                             \
        quantize_rows<DT_><<<row_blocks, kQThreads, 0, st>>>(x, groups, inner / 16, ldx, q, ldq, partial, np,  \
                                                             scale);                                           \
    else if (form == 2)                                                                                        \
        quantize_transpose<DT_><<<ttiles, kQThreads, 0, st>>>(x, outer, inner, ldx, q, ldq, partial, np,       \
                                                              scale);                                          \
    else if (any)                                                                                              \
        quantize_tiles<DT_><<<tiles, kQThreads, 0, st>>>(x, rows, cols, ldx, x_col, q, ldq, q_col, partial,    \
                                                         np, scale);
    switch (dtype) {
        case DT_F32: SKG_QUANT(DT_F32) break;
        case DT_BF16: SKG_QUANT(DT_BF16) break;
        case DT_F16: SKG_QUANT(DT_F16) break;
        default:
            return int(hipErrorInvalidValue);
    }
#undef SKG_QUANT
    return int(hipGetLastError());
}

}  // namespace skg
