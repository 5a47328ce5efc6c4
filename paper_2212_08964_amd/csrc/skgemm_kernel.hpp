// Persistent Stream-K GEMM kernels for gfx950 (CDNA4).
//
// One kernel template covers the data-parallel, basic Stream-K and hybrid
// schedules (Work Decomposition Strategies section, basic Stream-K algorithm;
// Data-parallel Hybridization subsection): each workgroup walks its even share
// of MAC-loop iterations across tile seams, then (or first) its whole
// data-parallel tiles.  A segment that does not start its tile publishes an
// FP32 partial tile and a ready flag; the segment holding the tile's k = 0
// iteration adds the partials of the following workgroups in ascending order
// and writes C, so results are deterministic for a fixed plan.
//
// MAC loop (the MacLoop subroutine): a WM x WN grid of wave64 wavefronts
// (2 x 2 for the FP32 128x128 tile, 2 x 4 for the 256x256 16-bit and FP8
// tiles, so no lane holds more than 128 FP32 accumulators).  Each k-iteration
// moves a BM x BK slab of A and a BK x BN slab of B straight from global
// memory into LDS with buffer loads that write LDS directly (no register
// staging); two LDS stages alternate so the next slab is in flight while the
// MFMAs consume the current one.  Each wave accumulates its (BM/WM) x (BN/WN)
// block with 32x32 MFMA instructions into FP32 registers.
//
// LDS layouts (no padding; 16-byte chunks XOR-swizzled per row so that the
// fragment reads of one instruction fall on distinct banks):
//  * K-contiguous operand: [rows][128 bytes of k]; chunk c of row r sits at
//    position c ^ (r mod 8) ^ ((r / 8) mod 2), so the 16-byte reads of 16
//    consecutive rows (one LDS cycle of 64 banks) touch distinct banks.
//  * MN-contiguous operand: [k][512 bytes of rows]; chunk c of row k sits at
//    position c ^ 4 (k mod 4) for 16-bit types (read with the LDS transpose
//    read, four k of one column per lane) and c ^ 8 ((k / 4) mod 2) for FP32
//    (read with plain 4-byte reads).

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "skgemm_internal.h"

namespace skg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

// Tile per input type and variant, and the wave grid that covers it (WM x WN
// wavefronts).  Variant 1 is the small 16-bit or FP8 tile (cheaper partial
// tiles and epilogues for small, memory-bound problems; two workgroups per
// CU); variant 2 the small 16-bit tile on eight waves (two per SIMD from one
// workgroup: shorter iterations when a CU holds one workgroup, longer when it
// holds two).
template <int DT, int V> struct Cfg;
// NS is the number of LDS stages of the MAC-loop pipeline (NS - 1 k-slabs in
// flight while one is consumed).
template <> struct Cfg<DT_F32, 0> { static constexpr int EB = 4, BM = kTileF32.bm, BN = kTileF32.bn, BK = kTileF32.bk, WM = 2, WN = 2, NS = kTileF32.ns; };
template <> struct Cfg<DT_F16, 0> { static constexpr int EB = 2, BM = kTile16.bm, BN = kTile16.bn, BK = kTile16.bk, WM = 2, WN = 4, NS = kTile16.ns; static constexpr bool PRIO = true; };
template <> struct Cfg<DT_BF16, 0> { static constexpr int EB = 2, BM = kTile16.bm, BN = kTile16.bn, BK = kTile16.bk, WM = 2, WN = 4, NS = kTile16.ns; static constexpr bool PRIO = true; };
template <> struct Cfg<DT_F8, 0> { static constexpr int EB = 1, BM = kTileF8.bm, BN = kTileF8.bn, BK = kTileF8.bk, WM = 2, WN = 4, NS = kTileF8.ns; };
template <> struct Cfg<DT_F8, 1> { static constexpr int EB = 1, BM = kTileF8S.bm, BN = kTileF8S.bn, BK = kTileF8S.bk, WM = 2, WN = 2, NS = kTileF8S.ns; };
template <> struct Cfg<DT_F64, 0> { static constexpr int EB = 8, BM = kTileF64.bm, BN = kTileF64.bn, BK = kTileF64.bk, WM = 2, WN = 2, NS = kTileF64.ns; };
template <> struct Cfg<DT_F64, 1> { static constexpr int EB = 8, BM = kTileF64L.bm, BN = kTileF64L.bn, BK = kTileF64L.bk, WM = 2, WN = 2, NS = kTileF64L.ns; };
template <> struct Cfg<DT_F16, 1> { static constexpr int EB = 2, BM = kTile16S.bm, BN = kTile16S.bn, BK = kTile16S.bk, WM = 2, WN = 2, NS = kTile16S.ns; };
template <> struct Cfg<DT_BF16, 1> { static constexpr int EB = 2, BM = kTile16S.bm, BN = kTile16S.bn, BK = kTile16S.bk, WM = 2, WN = 2, NS = kTile16S.ns; };
template <> struct Cfg<DT_F16, 2> { static constexpr int EB = 2, BM = kTile16S.bm, BN = kTile16S.bn, BK = kTile16S.bk, WM = 2, WN = 4, NS = kTile16S.ns; };
template <> struct Cfg<DT_BF16, 2> { static constexpr int EB = 2, BM = kTile16S.bm, BN = kTile16S.bn, BK = kTile16S.bk, WM = 2, WN = 4, NS = kTile16S.ns; };
// The same eight-wave tile on three LDS stages (96 KiB: one workgroup per
// CU), so two k-slabs are in flight while one is consumed: a lone workgroup
// on its CU then hides the load latency the two-stage pipeline exposes.  The
// register budget stays that of two workgroups per CU.
template <> struct Cfg<DT_F16, 8> { static constexpr int EB = 2, BM = kTile16D.bm, BN = kTile16D.bn, BK = kTile16D.bk, WM = 2, WN = 4, NS = kTile16D.ns, WPE = 4; };
template <> struct Cfg<DT_BF16, 8> { static constexpr int EB = 2, BM = kTile16D.bm, BN = kTile16D.bn, BK = kTile16D.bk, WM = 2, WN = 4, NS = kTile16D.ns, WPE = 4; };
// Skinny 16-bit tile for problems of at most 64 rows: four waves side by side
// over 256 columns (64x64 each), so a short A panel is padded to 64 rows, not
// 128 or 256.
template <> struct Cfg<DT_F16, 5> { static constexpr int EB = 2, BM = kTile16K.bm, BN = kTile16K.bn, BK = kTile16K.bk, WM = 1, WN = 4, NS = kTile16K.ns; };
template <> struct Cfg<DT_BF16, 5> { static constexpr int EB = 2, BM = kTile16K.bm, BN = kTile16K.bn, BK = kTile16K.bk, WM = 1, WN = 4, NS = kTile16K.ns; };
// Its transpose for problems of at most 64 columns (and convolutions with at
// most 64 output channels): four waves stacked over 256 rows.
template <> struct Cfg<DT_F16, 6> { static constexpr int EB = 2, BM = kTile16T.bm, BN = kTile16T.bn, BK = kTile16T.bk, WM = 4, WN = 1, NS = kTile16T.ns; };
template <> struct Cfg<DT_BF16, 6> { static constexpr int EB = 2, BM = kTile16T.bm, BN = kTile16T.bn, BK = kTile16T.bk, WM = 4, WN = 1, NS = kTile16T.ns; };
// Implicit-GEMM convolution: the tiles of variants 0 and 1 with A gathered
// from the NHWC input (CONV).
template <> struct Cfg<DT_F16, 3> : Cfg<DT_F16, 0> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_BF16, 3> : Cfg<DT_BF16, 0> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_F16, 4> : Cfg<DT_F16, 1> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_BF16, 4> : Cfg<DT_BF16, 1> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_F16, 7> : Cfg<DT_F16, 6> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_BF16, 7> : Cfg<DT_BF16, 6> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_F16, 9> : Cfg<DT_F16, 8> { static constexpr bool CONV = true; };
template <> struct Cfg<DT_BF16, 9> : Cfg<DT_BF16, 8> { static constexpr bool CONV = true; };

// Optional tile traits: PRIO raises the waves' priority through the MFMA
// section of each k-slab; WPE overrides the waves per SIMD the register
// budget is sized for.
template <class C, class = void> struct PrioOf { static constexpr bool value = false; };
template <class C> struct PrioOf<C, std::void_t<decltype(C::PRIO)>> { static constexpr bool value = C::PRIO; };
template <class C, class = void> struct ConvOf { static constexpr bool value = false; };
template <class C> struct ConvOf<C, std::void_t<decltype(C::CONV)>> { static constexpr bool value = C::CONV; };

template <int DT, int V>
constexpr int kThreadsOf = 64 * Cfg<DT, V>::WM * Cfg<DT, V>::WN;

// Waves per SIMD the register budget must allow: two workgroups per CU for
// the 4-wave tiles (the 8-wave tiles get two waves per SIMD from one, and the
// 8-wave small tile two workgroups); three for the 64x64 FP64 tile, whose
// accumulators take a quarter of the others', two for the 128x128 one.
template <class C, class = void> struct WpeOf { static constexpr int value = 0; };
template <class C> struct WpeOf<C, std::void_t<decltype(C::WPE)>> { static constexpr int value = C::WPE; };
template <int DT, int V>
constexpr int kWavesPerEU = WpeOf<Cfg<DT, V>>::value ? WpeOf<Cfg<DT, V>>::value
                            : DT == DT_F64 ? (V == 1 ? 2 : 3) : V == 2 ? 4 : 2;

// Buffer descriptor word 3 for untyped buffer loads on gfx9-family targets.
constexpr int kBufferFlags = 0x00020000;

__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// 32-bit LDS address of an LDS location (wave-uniform here).
__device__ __forceinline__ uint32_t lds_addr(unsigned char* p) {
    lds_void* q = (lds_void*)p;      // generic -> LDS address space (a C-style cast is required)
    return uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(size_t(q)))));
}

// One 16-byte-per-lane buffer load that writes LDS directly: lane i's chunk
// lands at LDS address m0 + 16 i; out-of-range offsets read as zero.  Issued
// as inline assembly so that the compiler's own wait-count bookkeeping does
// not see it: across the pipeline loop's back edge it cannot tell which LDS
// stage a load in flight targets and would drain all of them; the pipeline
// waits for its slabs itself (vmcnt, oldest first).  m0 is set here and used
// by nothing else in these kernels.
__device__ __forceinline__ void dma16(const i32x4& desc, uint32_t voff, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tbuffer_load_dwordx4 %0, %1, 0 offen lds"
                 :
                 : "v"(voff), "s"(desc), "s"(lds)
                 : "memory");
}

// Workgroup barrier between pipeline steps, without the memory fence of
// __syncthreads (which would also wait for the slab loads still in flight to
// the other stages).  Each wave's LDS accesses have completed (its fragment
// reads, and the slab loads it waited for explicitly) before it arrives.
__device__ __forceinline__ void step_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Values that are the same in every lane but reach the compiler through
// vector registers (a grouped launch reads its problem table with vector
// loads) are moved to scalar registers, so that buffer descriptors built from
// them stay scalar: a descriptor in vector registers forces a loop over the
// distinct lane values around every buffer load.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(x))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(x) >> 32))));
    return int64_t((uint64_t(hi) << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* unip(T* p) { return reinterpret_cast<T*>(uni64(reinterpret_cast<int64_t>(p))); }
__device__ __forceinline__ float unif(float x) { return __builtin_bit_cast(float, uni(__builtin_bit_cast(int, x))); }

// A copy of x the compiler cannot see through.  Per-lane addresses derived
// from the thread index are re-derived from such a copy where they are used,
// so they are not hoisted to the kernel's start and kept live (in registers
// the MAC loop's accumulators need) across every loop in between.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// ------------------------------------------------------------------ slab loads

// Position swizzle of a row of a slab in LDS (see the layout note above).
template <int EB, bool KC, int ROWB>
__device__ __forceinline__ int swz(int row) {
    if constexpr (KC && ROWB == 128) return (row & 7) ^ ((row >> 3) & 1);
    else if constexpr (KC) return (row >> 2) & 3;          // 64-byte rows: 4 chunks
    else if constexpr (EB == 4) return 8 * ((row >> 2) & 1);
    else return 4 * (row & 3);
}

// One operand's slab of a k-iteration: R rows of the output dimension by BK.
// The workgroup's waves split the slab's LDS image into 1 KiB blocks (64 lanes
// x 16 bytes); each lane fetches the global chunk whose swizzled position is
// its slot in the block.  Loads go through a buffer descriptor rebased at
// every k-iteration, so a lane keeps only 32-bit offsets, and the hardware
// returns zero for bytes past the end of the operand (rows beyond M or N of a
// K-contiguous operand, k beyond K of an MN-contiguous one).  In the checked
// form (the slabs that need it, see mac_loop) chunks that reach past the
// inner edge of a row (k beyond K, or columns beyond M or N) are skipped by
// the wide load (offset forced out of range: zero, no memory access) and,
// where partly inside, reloaded element by element.
template <int EB, int R, int BK, bool KC, int THREADS>
struct Slab {
    static constexpr int VE = 16 / EB;
    static constexpr int ROWB = KC ? BK * EB : R * EB;      // LDS row bytes
    static constexpr int BYTES = KC ? R * ROWB : BK * ROWB;
    static constexpr int NW = THREADS / 64;
    static constexpr int BLOCKS = BYTES / 1024;
    static constexpr int PER_WAVE = BLOCKS / NW;
    static_assert(!KC || BK * EB == 128 || BK * EB == 64, "K-contiguous slab rows must be 64 or 128 bytes");
    static_assert(KC || ROWB == 1024 || ROWB == 512 || ROWB == 256,
                  "MN-contiguous slab rows must be 256, 512 or 1024 bytes");
    static_assert(BLOCKS % NW == 0, "slab must split evenly over the waves");

    uint32_t voff[PER_WAVE];     // byte offset of the lane's chunk from the slab origin
    const unsigned char* base;   // operand address of (outer o0, k of the first iteration)
    int64_t bytes;               // operand bytes from base to its end
    int64_t step;                // bytes between consecutive k-iterations

    __device__ __forceinline__ void init(const void* X, int64_t ld, int o0, int dout, int kbeg, int K,
                                         int tid) {
        const int k0 = kbeg * BK;
        const unsigned char* p = reinterpret_cast<const unsigned char*>(X);
        if constexpr (KC) {
            base = p + ((int64_t)o0 * ld + k0) * EB;
            bytes = ((int64_t)(dout - o0 - 1) * ld + (K - k0)) * EB;
            step = BK * EB;
        } else {
            base = p + ((int64_t)k0 * ld + o0) * EB;
            bytes = ((int64_t)(K - k0 - 1) * ld + (dout - o0)) * EB;
            step = (int64_t)BK * ld * EB;
        }
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            const int row = chunk_row(j, tid);
            voff[j] = uint32_t(row) * uint32_t(ld * EB) + uint32_t(chunk_col(j, tid) * 16);
        }
    }

    // Slab row and (unswizzled) 16-byte chunk index of the lane's chunk j.
    static __device__ __forceinline__ int chunk_row(int j, int tid) {
        return (((tid >> 6) + j * NW) * 1024 + (tid & 63) * 16) / ROWB;
    }
    static __device__ __forceinline__ int chunk_col(int j, int tid) {
        const int pos = ((tid >> 6) + j * NW) * 1024 + (tid & 63) * 16;
        return ((pos % ROWB) >> 4) ^ swz<EB, KC, ROWB>(pos / ROWB);
    }

    __device__ __forceinline__ int nrec(int it) const {
        const int64_t left = bytes - (int64_t)it * step;
        return left <= 0 ? 0 : (left > 0x7fffffff ? 0x7fffffff : int(left));
    }

    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int it) const {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(base + (int64_t)it * step), (short)0,
                                                 nrec(it), kBufferFlags);
    }

    // The same descriptor as four scalar words (base, stride 0, records, flags).
    __device__ __forceinline__ i32x4 desc(int it) const {
        const uint64_t addr = reinterpret_cast<uint64_t>(base + (int64_t)it * step);
        return i32x4{uni(int(uint32_t(addr))), uni(int(uint32_t(addr >> 32) & 0xffffu)), uni(nrec(it)),
                     kBufferFlags};
    }

    // Elements of the lane's chunk j inside the inner edge (VE when not at the edge).
    __device__ __forceinline__ int keep(int j, bool tail, int lim, int tid) const {
        return tail ? min(max(lim - chunk_col(j, tid) * VE, 0), VE) : VE;
    }

    // A chunk that reaches past the inner edge but whose 16 bytes all lie
    // inside the buffer range (nr bytes from the slab origin) is loaded whole:
    // the bytes past the edge belong to the rest of the row (or the gap up to
    // the leading dimension, or the next row) and are cleared once the chunk
    // has landed.  Only a chunk that reaches past the operand's end needs the
    // element-by-element path.
    __device__ __forceinline__ bool whole(int j, uint32_t nr) const { return voff[j] + 16u <= nr; }

    // Issue the direct-to-LDS loads of iteration `it` (counted from kbeg), whose
    // first k is k0, into the stage at `lds`.  EDGE = false: the caller knows
    // the slab is wholly inside the inner edge (no per-chunk checks).
    template <bool EDGE>
    __device__ __forceinline__ void issue(int it, int k0, int K, int o0, int dout, unsigned char* lds,
                                          int tid) const {
        const i32x4 d = desc(it);
        const bool tail = EDGE && (KC ? (k0 + BK > K) : (o0 + R > dout));
        const int lim = KC ? (K - k0) : (dout - o0);
        const int w = uni(tid >> 6);
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            uint32_t off = voff[j];
            if constexpr (EDGE) {
                const int kp = keep(j, tail, lim, tid);
                if (kp == 0 || (kp < VE && !whole(j, uint32_t(d[2])))) off = 0x80000000u;
            }
            dma16(d, off, lds_addr(lds + (w + j * NW) * 1024));
        }
    }

    // After the stage's loads have landed: clear the bytes past the edge of
    // the partly-inside chunks that were loaded whole, and write the others
    // element by element.
    __device__ __forceinline__ void fix_edge(int it, int k0, int K, int o0, int dout, unsigned char* lds,
                                             int tid) const {
        const bool tail = KC ? (k0 + BK > K) : (o0 + R > dout);
        if (!tail) return;
        tid = opaque(tid);   // recompute the chunk positions here rather than keep issue()'s live
        const int lim = KC ? (K - k0) : (dout - o0);
        const uint32_t nr = uint32_t(uni(nrec(it)));
        const int lane = tid & 63, w = tid >> 6;
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            const int kp = keep(j, tail, lim, tid);
            // a chunk that starts past the operand's end has landed as zeros
            if (kp > 0 && kp < VE && voff[j] < nr) {
                unsigned char* dst = lds + (w + j * NW) * 1024 + lane * 16;
                if (whole(j, nr)) {
                    u32x4 v = *reinterpret_cast<const u32x4*>(dst);
                    const int nb = kp * EB;   // bytes inside the edge
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int kb = min(max(nb - 4 * q, 0), 4);
                        v[q] &= kb == 4 ? 0xffffffffu : (1u << (8 * kb)) - 1u;
                    }
                    *reinterpret_cast<u32x4*>(dst) = v;
                    continue;
                }
                // Element by element, in a loop that is not unrolled: this
                // runs only for chunks that straddle the operand's end, and
                // an unrolled form needs enough registers to push the
                // accumulators out to scratch.  Elements past the edge are
                // loaded too (zero past the operand's end) and replaced by
                // zero.
                const __amdgpu_buffer_rsrc_t rs = rsrc(it);
                const int off = int(voff[j]);
#pragma unroll 1
                for (int e = 0; e < VE; ++e) {
                    // the loads return raw bits (unsigned integers of the element's width)
                    if constexpr (EB == 8) {
                        const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 8 * e, 0, 0);
                        const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 8 * e + 4, 0, 0);
                        *reinterpret_cast<uint32_t*>(dst + 8 * e) = e < kp ? lo : 0u;
                        *reinterpret_cast<uint32_t*>(dst + 8 * e + 4) = e < kp ? hi : 0u;
                    } else if constexpr (EB == 4) {
                        const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * e, 0, 0);
                        *reinterpret_cast<uint32_t*>(dst + 4 * e) = e < kp ? x : 0u;
                    } else if constexpr (EB == 2) {
                        const uint16_t x = __builtin_amdgcn_raw_buffer_load_b16(rs, off + 2 * e, 0, 0);
                        *reinterpret_cast<uint16_t*>(dst + 2 * e) = e < kp ? x : uint16_t(0);
                    } else {
                        const uint8_t x = __builtin_amdgcn_raw_buffer_load_b8(rs, off + e, 0, 0);
                        dst[e] = e < kp ? x : uint8_t(0);
                    }
                }
            }
        }
    }
};

// The A slab of an implicit-GEMM convolution: R output pixels (GEMM rows) by
// BK reduction indices, laid out in LDS as a K-contiguous slab.  Every slab
// lies in one filter tap (r, s) and covers BK consecutive input channels
// (the planner requires C to be a multiple of BK), so a lane's 16-byte chunk
// is 8 consecutive channels of one input pixel: one direct-to-LDS load from
// the pixel's address, or zero (offset out of the buffer range) when the
// pixel lies in the padding or the row is past the last output pixel.
template <int EB, int R, int BK, int THREADS>
struct ConvSlab {
    static constexpr int VE = 16 / EB;
    static constexpr int ROWB = BK * EB;
    static constexpr int BYTES = R * ROWB;
    static constexpr int NW = THREADS / 64;
    static constexpr int BLOCKS = BYTES / 1024;
    static constexpr int PER_WAVE = BLOCKS / NW;
    static_assert(ROWB == 128 && BLOCKS % NW == 0, "convolution slabs: 128-byte rows split evenly over the waves");
    using S_ = Slab<EB, R, BK, true, THREADS>;   // the same chunk placement as a K-contiguous GEMM slab

    int hb[PER_WAVE], wb[PER_WAVE], ib[PER_WAVE];   // per chunk: first input row / column of the window, image * H
    const unsigned char* x;
    uint32_t bytes;
    int H, W, C, S, dil_h, dil_w;

    // The chunk rows' output pixels (rows past dout are never inside the image).
    __device__ __forceinline__ void init_conv(const ConvArgs& cv, const void* X, int o0, int dout, int tid) {
        x = reinterpret_cast<const unsigned char*>(X);
        H = uni(cv.h);
        W = uni(cv.w);
        C = uni(cv.c);
        S = uni(cv.s);
        dil_h = uni(cv.dil_h);
        dil_w = uni(cv.dil_w);
        const int P = uni(cv.p), Q = uni(cv.q), sh = uni(cv.str_h), sw = uni(cv.str_w);
        const int ph = uni(cv.pad_h), pw = uni(cv.pad_w);
        bytes = uint32_t(uni(int(int64_t(uni(cv.n)) * H * W * C * EB)));
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            const int m = o0 + S_::chunk_row(j, tid);
            const int pq = P * Q;
            const int img = m / pq, rem = m - img * pq, pp = rem / Q, qq = rem - pp * Q;
            const bool in = m < dout;
            hb[j] = in ? pp * sh - ph : -(1 << 30);   // never inside the image
            wb[j] = in ? qq * sw - pw : 0;
            ib[j] = in ? img * H : 0;
        }
    }

    // Slab of reduction indices [k0, k0 + BK): filter tap k0 / C, channels k0 mod C on.
    template <bool EDGE>
    __device__ __forceinline__ void issue(int, int k0, int, int, int, unsigned char* lds, int tid) const {
        const int rs = k0 / C, c0 = k0 - rs * C;
        const int r = rs / S, s = rs - r * S;
        const i32x4 d = {uni(int(uint32_t(reinterpret_cast<uint64_t>(x)))),
                         uni(int(uint32_t(reinterpret_cast<uint64_t>(x) >> 32) & 0xffffu)), int(bytes), kBufferFlags};
        const int w = uni(tid >> 6);
#pragma unroll
        for (int j = 0; j < PER_WAVE; ++j) {
            const int h = hb[j] + r * dil_h, ww = wb[j] + s * dil_w;
            uint32_t off = 0x80000000u;
            if (uint32_t(h) < uint32_t(H) && uint32_t(ww) < uint32_t(W))
                off = uint32_t((((ib[j] + h) * W + ww) * C + c0 + S_::chunk_col(j, tid) * VE) * EB);
            dma16(d, off, lds_addr(lds + (w + j * NW) * 1024));
        }
    }

    // Convolution slabs have no ragged inner edge: nothing to fix.
    __device__ __forceinline__ void fix_edge(int, int, int, int, int, unsigned char*, int) const {}
};

// ------------------------------------------------------------------ LDS fragment reads

// 16 bytes = 8 k-values of one row of a K-contiguous slab, chunk q (0..7).
template <int ROWB>
__device__ __forceinline__ u32x4 lds_row_chunk(const unsigned char* lds, int row, int q) {
    return *reinterpret_cast<const u32x4*>(lds + row * ROWB + ((q ^ swz<2, true, ROWB>(row)) << 4));
}

// Byte address of element (k, col) of an MN-contiguous slab with ROWB-byte rows.
template <int EB, int ROWB>
__device__ __forceinline__ int mn_addr(int k, int col) {
    constexpr int VE = 16 / EB;
    return k * ROWB + (((col / VE) ^ swz<EB, false, ROWB>(k)) << 4) + (col % VE) * EB;
}

// Eight consecutive k (kb .. kb+7) of column (ob + lane % 32) of an MN-contiguous
// 16-bit slab, via two LDS transpose reads of four k each.  Within each group
// of 16 lanes the transpose read returns, to lane i, element i mod 4 of the
// 8-byte words fetched by lanes 4e + i / 4 (e = 0..3); so lane j of the group
// fetches row kb + j / 4, columns 4 (j mod 4) .. +3 of its 16-column half.
template <int ROWB>
__device__ __forceinline__ u32x4 lds_tr16(const unsigned char* lds, int kb, int ob, int lane) {
    const int sub = lane & 15, h = lane >> 4;
    const int col = ob + 16 * (h & 1) + 4 * (sub & 3);
    const int k = kb + (sub >> 2);
    typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
    lds_i16x4* p0 = (lds_i16x4*)(lds + mn_addr<2, ROWB>(k, col));
    lds_i16x4* p1 = (lds_i16x4*)(lds + mn_addr<2, ROWB>(k + 4, col));
    const i16x4 v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(p0);
    const i16x4 v1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(p1);
    const u32x2 a = __builtin_bit_cast(u32x2, v0);
    const u32x2 b = __builtin_bit_cast(u32x2, v1);
    return u32x4{a.x, a.y, b.x, b.y};
}

// ------------------------------------------------------------------ MFMA

template <int DT>
__device__ __forceinline__ f32x16 mfma16(const u32x4& a, const u32x4& b, const f32x16& c) {
    if constexpr (DT == DT_BF16) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
}

// ------------------------------------------------------------------ output conversion

// Round to nearest even with the hardware conversions (v_cvt_pk_bf16_f32 for
// bfloat16; NaN stays NaN).  A software rounding with a NaN branch made every
// element a divergent branch in the epilogue.
template <int OUT>
__device__ __forceinline__ uint16_t f32_to_half(float x) {
    if constexpr (OUT == DT_BF16) return __builtin_bit_cast(uint16_t, __bf16(x));
    else return __builtin_bit_cast(uint16_t, _Float16(x));
}

// Two values, packed low then high.
template <int OUT>
__device__ __forceinline__ uint32_t f32x2_to_half2(float x0, float x1) {
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    if constexpr (OUT == DT_BF16) {
        typedef __bf16 h2_t __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{x0, x1}, h2_t));
    } else {
        typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{x0, x1}, h2_t));
    }
}

template <int OUT>
__device__ __forceinline__ float half_to_f32(uint16_t h) {
    if constexpr (OUT == DT_BF16) return __builtin_bit_cast(float, uint32_t(h) << 16);
    else return float(__builtin_bit_cast(_Float16, h));
}

// C is reached through global-address-space pointers: generic (flat) memory
// instructions also count against the LDS wait counter, so every LDS read of
// the epilogue would wait for the previous band's C stores to complete.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> global(void* p) { return (gptr<T>)p; }

template <int OUT>
__device__ __forceinline__ float load_c1(void* C, int64_t off) {
    if constexpr (OUT == DT_F32) return global<float>(C)[off];
    else return half_to_f32<OUT>(global<uint16_t>(C)[off]);
}

template <int OUT>
__device__ __forceinline__ void store_c1(void* C, int64_t off, float v) {
    if constexpr (OUT == DT_F32) global<float>(C)[off] = v;
    else global<uint16_t>(C)[off] = f32_to_half<OUT>(v);
}

// ------------------------------------------------------------------ the kernel

// The problem a segment belongs to (the whole launch for a single GEMM, one
// table entry for a grouped launch).
struct Prob {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    int M, N, K, tn, ipt;
    float alpha, beta;
    int raster;          // tile rows per raster group (1 = plain row-major)
    ConvArgs conv;       // implicit-GEMM convolution (A gathered from its input), else unused
};

__device__ __forceinline__ Prob uniform(const Prob& p) {
    return Prob{unip(p.A), unip(p.B), unip(p.C), uni64(p.lda), uni64(p.ldb), uni64(p.ldc), uni(p.M), uni(p.N),
                uni(p.K), uni(p.tn), uni(p.ipt), unif(p.alpha), unif(p.beta), uni(p.raster), p.conv};
}

// The problem's fields as scalars the compiler cannot see through: values
// derived from them are re-derived per segment rather than hoisted out of the
// segment loop and kept live across the MAC loop.
template <class T>
__device__ __forceinline__ T opaque_s(T x) {
    if constexpr (sizeof(T) == 8) {
        uint64_t u = __builtin_bit_cast(uint64_t, x);
        asm volatile("" : "+s"(u));
        return __builtin_bit_cast(T, u);
    } else {
        asm volatile("" : "+s"(x));
        return x;
    }
}

__device__ __forceinline__ Prob opaque_prob(const Prob& p) {
    return Prob{opaque_s(p.A), opaque_s(p.B), opaque_s(p.C), opaque_s(p.lda), opaque_s(p.ldb), opaque_s(p.ldc),
                opaque_s(p.M), opaque_s(p.N), opaque_s(p.K), opaque_s(p.tn), opaque_s(p.ipt), opaque_s(p.alpha),
                opaque_s(p.beta), opaque_s(p.raster), p.conv};
}

template <bool B, class T, class F> struct Pick { using type = T; };
template <class T, class F> struct Pick<false, T, F> { using type = F; };

// One FP64 element of a staged slab: K-contiguous rows of 16 doubles (chunk of
// two per 16 bytes, swizzled by row) or MN-contiguous rows of one k.
template <bool KC, int ROWB>
__device__ __forceinline__ double lds_f64(const unsigned char* lds, int outer, int k) {
    if constexpr (KC)
        return *reinterpret_cast<const double*>(lds + outer * ROWB + (((k >> 1) ^ swz<8, true, ROWB>(outer)) << 4) +
                                                (k & 1) * 8);
    else
        return *reinterpret_cast<const double*>(lds + mn_addr<8, ROWB>(k, outer));
}

template <int DT, bool AKC, bool BKC, int V>
struct Gemm {
    using C_ = Cfg<DT, V>;
    static constexpr int EB = C_::EB, BM = C_::BM, BN = C_::BN, BK = C_::BK;
    static constexpr int WM = C_::WM, WN = C_::WN, THREADS = 64 * WM * WN, NW = WM * WN;
    static constexpr int WTM = BM / WM, WTN = BN / WN;    // wave tile
    static constexpr int FM = WTM / 32, FN = WTN / 32;    // 32x32 MFMA blocks per wave
    static constexpr bool CONV = ConvOf<C_>::value;
    static_assert(!CONV || (AKC && BKC && (DT == DT_BF16 || DT == DT_F16)), "convolution: 16-bit, filters K-contiguous");
    using SA = typename Pick<CONV, ConvSlab<EB, BM, BK, THREADS>, Slab<EB, BM, BK, AKC, THREADS>>::type;
    using SB = Slab<EB, BN, BK, BKC, THREADS>;
    static constexpr int STAGE = SA::BYTES + SB::BYTES;
    static constexpr int NS = C_::NS;
    static_assert(NS >= 2 && NS * STAGE <= 160 * 1024, "LDS budget");
    // direct-to-LDS loads each thread issues per k-iteration
    static constexpr int LOADS = SA::PER_WAVE + SB::PER_WAVE;

    // The pipeline's LDS stages: NS separate objects, so that the compiler
    // can tell the stage being read from the stages being filled.  Named
    // members picked by compile-time index: a pointer array indexed in a loop
    // would be moved to LDS per thread by the compiler.
    struct Stages {
        unsigned char *s0, *s1, *s2, *s3, *s4;
        template <int J>
        __device__ __forceinline__ unsigned char* at() const {
            static_assert(J >= 0 && J < NS, "stage index");
            if constexpr (J == 0) return s0;
            else if constexpr (J == 1) return s1;
            else if constexpr (J == 2) return s2;
            else if constexpr (J == 3) return s3;
            else return s4;
        }
    };

    // FP32 accumulators: one 32x32 MFMA block per (i, j).  FP64: four 16x16
    // MFMA blocks per 32x32 block (q = 2 * row half + column half), so bands
    // and blocks cover the same rows and columns for every type.
    struct Acc32 { f32x16 v[FM][FN]; };
    struct Acc64 { f64x4 v[FM][FN][4]; };
    using Acc = typename Pick<DT == DT_F64, Acc64, Acc32>::type;
    // 16-byte chunks of one block's accumulators per lane (partial tiles are
    // stored and read in this fragment order)
    static constexpr int CPB = DT == DT_F64 ? 8 : 4;
    // floats per partial slot
    static constexpr int SLOT = DT == DT_F64 ? 2 * BM * BN : BM * BN;

    static __device__ __forceinline__ u32x4 acc_chunk(const Acc& acc, int i, int j, int r) {
        if constexpr (DT == DT_F64) {
            const f64x4& b = acc.v[i][j][r >> 1];
            const f64x2 v = (r & 1) ? f64x2{b[2], b[3]} : f64x2{b[0], b[1]};
            return __builtin_bit_cast(u32x4, v);
        } else {
            const f32x4 v = {acc.v[i][j][4 * r], acc.v[i][j][4 * r + 1], acc.v[i][j][4 * r + 2],
                             acc.v[i][j][4 * r + 3]};
            return __builtin_bit_cast(u32x4, v);
        }
    }

    // One block's worth of partial sums kept apart from the accumulators (the
    // running sum of the contributors ahead of this one in the split fix-up).
    struct Blk32 { f32x16 v; };
    struct Blk64 { f64x4 q[4]; };
    using Blk = typename Pick<DT == DT_F64, Blk64, Blk32>::type;

    // T chunk r = bits (first) or T chunk r += bits
    static __device__ __forceinline__ void blk_take_chunk(Blk& T, int r, const u32x4& bits, bool first) {
        if constexpr (DT == DT_F64) {
            const f64x2 v = __builtin_bit_cast(f64x2, bits);
            f64x4& b = T.q[r >> 1];
            const int o = (r & 1) * 2;
            b[o] = first ? v.x : b[o] + v.x;
            b[o + 1] = first ? v.y : b[o + 1] + v.y;
        } else {
            const f32x4 v = __builtin_bit_cast(f32x4, bits);
            T.v[4 * r] = first ? v.x : T.v[4 * r] + v.x;
            T.v[4 * r + 1] = first ? v.y : T.v[4 * r + 1] + v.y;
            T.v[4 * r + 2] = first ? v.z : T.v[4 * r + 2] + v.z;
            T.v[4 * r + 3] = first ? v.w : T.v[4 * r + 3] + v.w;
        }
    }

    // block (i, j) of acc = T + block (i, j)
    static __device__ __forceinline__ void acc_add_blk(Acc& acc, int i, int j, const Blk& T) {
        if constexpr (DT == DT_F64) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc.v[i][j][q] = T.q[q] + acc.v[i][j][q];
        } else {
            acc.v[i][j] = T.v + acc.v[i][j];
        }
    }

    static __device__ __forceinline__ void acc_add_chunk(Acc& acc, int i, int j, int r, const u32x4& bits) {
        if constexpr (DT == DT_F64) {
            const f64x2 v = __builtin_bit_cast(f64x2, bits);
            f64x4& b = acc.v[i][j][r >> 1];
            if (r & 1) {
                b[2] += v.x;
                b[3] += v.y;
            } else {
                b[0] += v.x;
                b[1] += v.y;
            }
        } else {
            const f32x4 v = __builtin_bit_cast(f32x4, bits);
            acc.v[i][j][4 * r] += v.x;
            acc.v[i][j][4 * r + 1] += v.y;
            acc.v[i][j][4 * r + 2] += v.z;
            acc.v[i][j][4 * r + 3] += v.w;
        }
    }

    // MFMAs over one staged k-slab.
    static __device__ __forceinline__ void compute(const unsigned char* As, const unsigned char* Bs,
                                                   Acc& acc, int wm, int wn, int lane) {
        const int g = lane >> 5, l32 = lane & 31;
        if constexpr (DT == DT_BF16 || DT == DT_F16) {
            // Fragments are double-buffered across the k16 steps: the reads of
            // step s+1 are interleaved between the MFMAs of step s, so LDS
            // latency hides behind matrix work instead of stalling it.
            constexpr int KS = BK / 16;
            u32x4 af[2][FM], bf[2][FN];
            auto load = [&](int s, int buf) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    if constexpr (AKC) af[buf][i] = lds_row_chunk<SA::ROWB>(As, wm * WTM + i * 32 + l32, 2 * s + g);
                    else af[buf][i] = lds_tr16<SA::ROWB>(As, 16 * s + 8 * g, wm * WTM + i * 32, lane);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (BKC) bf[buf][j] = lds_row_chunk<SB::ROWB>(Bs, wn * WTN + j * 32 + l32, 2 * s + g);
                    else bf[buf][j] = lds_tr16<SB::ROWB>(Bs, 16 * s + 8 * g, wn * WTN + j * 32, lane);
                }
            };
            // LDS reads per step: one per K-contiguous fragment, two per
            // transposed one
            constexpr int READS = FM * (AKC ? 1 : 2) + FN * (BKC ? 1 : 2);
            constexpr int MFMAS = FM * FN;
            load(0, 0);
            // PRIO (the 256x256 tile: two waves per SIMD from one workgroup):
            // a raised priority while a wave is in its MFMA section lets it
            // keep the matrix core busy ahead of the other wave's loads and
            // barrier (measured +1.5-2.5 % on large shapes; neutral on the
            // small tiles, which keep the default).
            if constexpr (PrioOf<C_>::value) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int cur = s & 1;
                // The reads of step s+1 are interleaved one by one between
                // the MFMAs of step s, which cover their latency; the group
                // barriers fix that order (MFMA, read, MFMA, read, ...) and
                // the closing barrier keeps the compiler from moving work
                // across steps.
                if (s + 1 < KS) load(s + 1, cur ^ 1);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc.v[i][j] = mfma16<DT>(af[cur][i], bf[cur][j], acc.v[i][j]);
                if (s + 1 < KS) {
#pragma unroll
                    for (int k = 0; k < READS || k < MFMAS; ++k) {
                        if (k < MFMAS) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
                        if (k < READS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (PrioOf<C_>::value) __builtin_amdgcn_s_setprio(0);
        } else if constexpr (DT == DT_F64) {
            // v_mfma_f64_16x16x4f64: lane l holds A[row l%16][k l/16] and
            // B[k l/16][col l%16] of the k4 step; each 32x32 block is four
            // 16x16 MFMA blocks.
            const int l16 = lane & 15, kq = lane >> 4;
#pragma unroll
            for (int s = 0; s < BK / 4; ++s) {
                const int k = 4 * s + kq;
                double af[FM][2], bf[FN][2];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int h = 0; h < 2; ++h) af[i][h] = lds_f64<AKC, SA::ROWB>(As, wm * WTM + i * 32 + h * 16 + l16, k);
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int h = 0; h < 2; ++h) bf[j][h] = lds_f64<BKC, SB::ROWB>(Bs, wn * WTN + j * 32 + h * 16 + l16, k);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc.v[i][j][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][q >> 1], bf[j][q & 1],
                                                                                 acc.v[i][j][q], 0, 0, 0);
            }
        } else if constexpr (DT == DT_F32) {
            // Lane group g handles k = 8c + 4g + u of step (c, u).
#pragma unroll
            for (int c = 0; c < BK / 8; ++c) {
                f32x4 af[FM], bf[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int row = wm * WTM + i * 32 + l32;
                    if constexpr (AKC) {
                        af[i] = __builtin_bit_cast(f32x4, lds_row_chunk<SA::ROWB>(As, row, 2 * c + g));
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            af[i][u] = *reinterpret_cast<const float*>(As + mn_addr<4, SA::ROWB>(8 * c + 4 * g + u, row));
                    }
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int col = wn * WTN + j * 32 + l32;
                    if constexpr (BKC) {
                        bf[j] = __builtin_bit_cast(f32x4, lds_row_chunk<SB::ROWB>(Bs, col, 2 * c + g));
                    } else {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            bf[j][u] = *reinterpret_cast<const float*>(Bs + mn_addr<4, SB::ROWB>(8 * c + 4 * g + u, col));
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc.v[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][u], bf[j][u], acc.v[i][j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            static_assert(AKC && BKC, "FP8 operands must be K-contiguous");
            // Lane group g handles k = 64s + 32g .. +31 of step s (two chunks).
            // Not unrolled, and B fragments for the step, then one A
            // fragment at a time: the fewest registers in flight.  Any spill
            // would make the kernel use scratch memory, and a kernel with
            // scratch pays a fixed cost of about 20 us per launch on this GPU.
#pragma unroll 1
            for (int s = 0; s < BK / 64; ++s) {
                i32x8 bf[FN];
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int row = wn * WTN + j * 32 + l32;
                    const u32x4 lo = lds_row_chunk<SB::ROWB>(Bs, row, 4 * s + 2 * g);
                    const u32x4 hi = lds_row_chunk<SB::ROWB>(Bs, row, 4 * s + 2 * g + 1);
                    bf[j] = i32x8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
                }
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int row = wm * WTM + i * 32 + l32;
                    const u32x4 lo = lds_row_chunk<SA::ROWB>(As, row, 4 * s + 2 * g);
                    const u32x4 hi = lds_row_chunk<SA::ROWB>(As, row, 4 * s + 2 * g + 1);
                    const i32x8 af = i32x8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y),
                                           int(hi.z), int(hi.w)};
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc.v[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            af, bf[j], acc.v[i][j], 0, 0, 0, 127, 0, 127);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // Output block of a tile index.  Tile indices run down a group of
    // `raster` tile rows before moving to the next column, so consecutive
    // tiles (the ones neighbouring workgroups work on at the same time) form
    // a compact block that shares A and B slabs in the L2 cache.  A bijection
    // of [0, tm*tn) for any raster >= 1; raster = 1 is row-major order.
    static __device__ __forceinline__ void tile_origin(const Prob& a, int tile, int& m0, int& n0) {
        const int tm = (a.M + BM - 1) / BM;
        const int rows = min(a.raster, tm);     // rows * tn <= tiles: no overflow
        const int span = rows * a.tn;
        const int grp = tile / span;
        const int first = grp * rows;
        const int gm = min(tm - first, rows);
        const int in = tile - grp * span;
        m0 = (first + in % gm) * BM;
        n0 = (in / gm) * BN;
    }

    // Wait until the k-slab after the current one has landed: at most `newer`
    // iterations' loads (issued after it) may still be in flight.
    template <int N>
    static __device__ __forceinline__ void wait_vmem_le() {
        static_assert(N >= 0 && N < 64, "vmcnt range");
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
    }
    static __device__ __forceinline__ void wait_slab(int newer) {
        if constexpr (NS >= 5)
            if (newer >= 3) return wait_vmem_le<LOADS * 3>();
        if constexpr (NS >= 4)
            if (newer >= 2) return wait_vmem_le<LOADS * 2>();
        if constexpr (NS >= 3)
            if (newer >= 1) return wait_vmem_le<LOADS>();
        wait_vmem();
    }

    // One step of the MAC loop, iteration it (stage `cur`): start the loads of
    // iteration it + NS - 1 into stage `nxt` (freed by iteration it - 1, which
    // every wave finished before the last barrier), run the MFMAs of `cur`,
    // wait for the slab of iteration it + 1 (stage `fix`) and synchronise.
    // Slabs of iterations from kedge on are loaded with per-chunk checks
    // against the operands' inner edges (and fixed up once they have landed);
    // the others lie wholly inside them.
    static __device__ __forceinline__ bool step(const Prob& a, const SA& sa, const SB& sb, int it, int kbeg,
                                                int kend, int kedge, int m0, int n0, unsigned char* cur,
                                                unsigned char* nxt, unsigned char* fix, Acc& acc, int tid) {
        const int lane = tid & 63, w = tid >> 6, wm = w / WN, wn = w % WN;
        const int ahead = it + NS - 1;
        if (ahead < kend) {
            if (ahead < kedge) {
                sa.template issue<false>(ahead - kbeg, ahead * BK, a.K, m0, a.M, nxt, tid);
                sb.template issue<false>(ahead - kbeg, ahead * BK, a.K, n0, a.N, nxt + SA::BYTES, tid);
            } else {
                sa.template issue<true>(ahead - kbeg, ahead * BK, a.K, m0, a.M, nxt, tid);
                sb.template issue<true>(ahead - kbeg, ahead * BK, a.K, n0, a.N, nxt + SA::BYTES, tid);
            }
        }
        compute(cur, cur + SA::BYTES, acc, wm, wn, lane);
        const bool more = it + 1 < kend;
        if (more) {
            wait_slab(min(NS - 2, kend - 2 - it));
            if (it + 1 >= kedge) {
                sa.fix_edge(it + 1 - kbeg, (it + 1) * BK, a.K, m0, a.M, fix, tid);
                sb.fix_edge(it + 1 - kbeg, (it + 1) * BK, a.K, n0, a.N, fix + SA::BYTES, tid);
            }
        }
        step_barrier();
        return more;
    }

    // Iterations kk + U (U = 0 .. NS-1) of the pipeline, each on its own
    // stage; false once the last iteration has been consumed.
    template <int... U>
    static __device__ __forceinline__ bool steps(const Prob& a, const SA& sa, const SB& sb, int kk, int kbeg,
                                                 int kend, int kedge, int m0, int n0, const Stages& st, Acc& acc,
                                                 int tid, std::integer_sequence<int, U...>) {
        return (step(a, sa, sb, kk + U, kbeg, kend, kedge, m0, n0, st.template at<U>(),
                     st.template at<(U + NS - 1) % NS>(), st.template at<(U + 1) % NS>(), acc, tid) &&
                ...);
    }

    // Slab kbeg + J into stage J, checked from kedge on.
    template <int J>
    static __device__ __forceinline__ void prologue_one(const Prob& a, const SA& sa, const SB& sb, int kbeg,
                                                        int kend, int kedge, int m0, int n0, const Stages& st,
                                                        int tid) {
        const int it = kbeg + J;
        if (it >= kend) return;
        if (it < kedge) {
            sa.template issue<false>(J, it * BK, a.K, m0, a.M, st.template at<J>(), tid);
            sb.template issue<false>(J, it * BK, a.K, n0, a.N, st.template at<J>() + SA::BYTES, tid);
        } else {
            sa.template issue<true>(J, it * BK, a.K, m0, a.M, st.template at<J>(), tid);
            sb.template issue<true>(J, it * BK, a.K, n0, a.N, st.template at<J>() + SA::BYTES, tid);
        }
    }

    // Prologue: slab kbeg + J into stage J (J = 0 .. NS-2).
    template <int... J>
    static __device__ __forceinline__ void prologue(const Prob& a, const SA& sa, const SB& sb, int kbeg, int kend,
                                                    int kedge, int m0, int n0, const Stages& st, int tid,
                                                    std::integer_sequence<int, J...>) {
        (prologue_one<J>(a, sa, sb, kbeg, kend, kedge, m0, n0, st, tid), ...);
    }

    // Iterations [kbeg, kend) of a tile: the first NS - 1 slabs are loaded
    // up front, then each step consumes one stage and refills the stage the
    // previous step consumed.  Iteration it uses stage (it - kbeg) mod NS.
    // Slabs of iterations from kedge on get per-chunk edge checks, inside the
    // same pipeline.
    static __device__ __forceinline__ void loop(const Prob& a, const Stages& st, int m0, int n0, int kbeg, int kend,
                                                int kedge, Acc& acc, int tid) {
        tid = opaque(tid);
        SA sa;
        SB sb;
        if constexpr (CONV) sa.init_conv(a.conv, a.A, m0, a.M, tid);
        else sa.init(a.A, a.lda, m0, a.M, kbeg, a.K, tid);
        sb.init(a.B, a.ldb, n0, a.N, kbeg, a.K, tid);
        __syncthreads();   // LDS may still be in use (previous epilogue or loop)
        prologue(a, sa, sb, kbeg, kend, kedge, m0, n0, st, tid, std::make_integer_sequence<int, NS - 1>{});
        wait_slab(min(NS - 2, kend - 1 - kbeg));
        if (kbeg >= kedge) {
            sa.fix_edge(0, kbeg * BK, a.K, m0, a.M, st.template at<0>(), tid);
            sb.fix_edge(0, kbeg * BK, a.K, n0, a.N, st.template at<0>() + SA::BYTES, tid);
        }
        step_barrier();
        for (int kk = kbeg;; kk += NS)
            if (!steps(a, sa, sb, kk, kbeg, kend, kedge, m0, n0, st, acc, tid, std::make_integer_sequence<int, NS>{}))
                return;
    }

    // MAC-loop iterations [klo, khi) of one tile into acc (zeroed first).
    // Only the tile's last k-iteration can need per-chunk checks: there a
    // K-contiguous operand's chunks may straddle k = K (the elements past it
    // belong to the next row and must read as zero), and an MN-contiguous
    // operand's chunk in row K-1 may straddle the operand's end (the whole
    // chunk would read as zero).  Every other slab is loaded with plain
    // 16-byte chunks: chunks past the M or N edge of an MN-contiguous operand
    // only feed rows or columns of the tile that are never written.
    static __device__ __forceinline__ void mac_loop(const Prob& a, const Stages& st, int tile, int klo, int khi,
                                                    Acc& acc, int tid) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if constexpr (DT == DT_F64) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc.v[i][j][q] = f64x4{0, 0, 0, 0};
                } else {
                    acc.v[i][j] = f32x16{0};
                }
            }
        if (klo >= khi) return;
        int m0, n0;
        tile_origin(a, tile, m0, n0);
        const int klast = (a.K + BK - 1) / BK - 1;
        const bool a_edge = !AKC && m0 + BM > a.M, b_edge = !BKC && n0 + BN > a.N;
        const bool check_last = ((AKC || BKC) && a.K % BK != 0) || a_edge || b_edge;
        // rows shorter than a chunk: chunks of earlier rows can reach the end too
        const bool check_all = (a_edge && a.lda * EB < 16) || (b_edge && a.ldb * EB < 16);
        const int kedge = check_all ? klo : check_last ? klast : khi;
        loop(a, st, m0, n0, klo, khi, kedge, acc, tid);
    }

    // Partial tiles are stored in fragment order: 16-byte chunk q of thread
    // tid at byte (q * THREADS + tid) * 16 of the slot, so each store
    // instruction of the workgroup writes THREADS * 16 bytes contiguously and
    // the reader uses the same mapping.
    //
    // The eight XCDs keep separate, non-coherent L2 caches, and the reader of a
    // partial usually runs on another XCD.  Partials and flags therefore move
    // with device-coherent (SC1) stores and loads, the cache policy the
    // compiler uses for agent-scope atomics: the data reaches the device
    // coherence point before the store completes, and the reader fetches it
    // from there, so neither side needs a whole-L2 write-back or invalidate
    // (which would also evict the A/B slabs of every workgroup on that XCD).
    static constexpr int kCoherent = 16;   // SC1 cache-policy bit

    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t slot_rsrc(float* slot) {
        return __builtin_amdgcn_make_buffer_rsrc(slot, (short)0, SLOT * 4, kBufferFlags);
    }

    // Output of 32 rows x W columns staged in `st` (FP32, rows of EPI_LD
    // floats): each lane converts eight consecutive columns of one row and
    // writes them with one store, predicated at the M and N edges.
    template <int OUT, int W>
    static __device__ __forceinline__ void write_band(const Prob& a, float s, const float* st, int row0, int col,
                                                      int ncol, int lane) {
        constexpr int LPR = W / 8;            // lanes per row
        constexpr int RPP = 64 / LPR;         // rows per pass
#pragma unroll
        for (int pass = 0; pass < 32 / RPP; ++pass) {
            const int rl = pass * RPP + lane / LPR;
            const int row = row0 + rl;
            const f32x4 lo = *reinterpret_cast<const f32x4*>(st + rl * EPI_LD + (lane % LPR) * 8);
            const f32x4 hi = *reinterpret_cast<const f32x4*>(st + rl * EPI_LD + (lane % LPR) * 8 + 4);
            const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            if (row < a.M && ncol > 0) {
                const int64_t off = (int64_t)row * a.ldc + col;
                if (ncol == 8) {
                    if constexpr (OUT == DT_F32) {
                        gptr<f32x4> cp = (gptr<f32x4>)(global<float>(a.C) + off);
                        f32x4 o0 = {v[0], v[1], v[2], v[3]}, o1 = {v[4], v[5], v[6], v[7]};
                        o0 *= s;
                        o1 *= s;
                        if (a.beta != 0.0f) {
                            o0 += a.beta * cp[0];
                            o1 += a.beta * cp[1];
                        }
                        cp[0] = o0;
                        cp[1] = o1;
                    } else {
                        gptr<u32x4> cp = (gptr<u32x4>)(global<uint16_t>(a.C) + off);
                        float cin[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                        if (a.beta != 0.0f) {
                            const u32x4 cv = *cp;
#pragma unroll
                            for (int e = 0; e < 8; ++e)
                                cin[e] = half_to_f32<OUT>(uint16_t(cv[e >> 1] >> (16 * (e & 1))));
                        }
                        u32x4 o;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float x0 = s * v[2 * e] + a.beta * cin[2 * e];
                            const float x1 = s * v[2 * e + 1] + a.beta * cin[2 * e + 1];
                            o[e] = f32x2_to_half2<OUT>(x0, x1);
                        }
                        *cp = o;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        if (e < ncol) {
                            float x = s * v[e];
                            if (a.beta != 0.0f) x += a.beta * load_c1<OUT>(a.C, off + e);
                            store_c1<OUT>(a.C, off + e, x);
                        }
                    }
                }
            }
        }
    }

    // FP64 output straight from the MFMA layout: lane l holds column l % 16
    // of rows l / 16 + 4 e of each 16x16 block, so every store instruction
    // writes four runs of 128 contiguous bytes.  Predicated at the M and N edges.
    static __device__ __forceinline__ void write_block_f64(const Prob& a, double s, const Acc& acc, int i, int j,
                                                           int m0, int n0, int lane) {
        if constexpr (DT == DT_F64) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = n0 + j * 32 + (q & 1) * 16 + (lane & 15);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = m0 + i * 32 + (q >> 1) * 16 + (lane >> 4) + 4 * e;
                    if (row < a.M && col < a.N) {
                        gptr<double> cp = global<double>(a.C) + ((int64_t)row * a.ldc + col);
                        double x = s * acc.v[i][j][q][e];
                        if (a.beta != 0.0f) x += double(a.beta) * *cp;
                        *cp = x;
                    }
                }
            }
        }
    }

    // How a segment's accumulators leave the registers: units of one 32x32
    // block (FM x FN per wave, unit u = i * FN + j) go out in two passes.
    // Pass 1 stores the units in `store_mask` into this workgroup's slot
    // (coherent stores, fragment order: 16-byte chunk q of thread tid at byte
    // (q * THREADS + tid) * 16) and raises the ready-flag words in
    // `flag_words` (bit f: word f of this workgroup's flag line).  Pass 2
    // reduces and writes the units in `fin_mask`: it waits for word `fw` of
    // the flags of peers lo .. hi (this workgroup excluded) and sums every
    // unit over lo .. hi in ascending order, its own accumulators in its own
    // place (the peers ahead of it are summed apart first, then added to
    // them), and writes the unit through the epilogue, C = alpha * s_A * s_B *
    // acc + beta * C; then it clears the words it waited on.  The next peer's
    // copy is loaded while the current one is added.
    //
    //   partial share (owner fix-up):  store all units, raise word 0
    //   owner (owner fix-up):          reduce all units, peers wg+1 .. last, word 0
    //   whole tile:                    write all units
    //   split fix-up, contributor c:   the first R = min(s, REDUCERS) contributors
    //                                  reduce: whole bands (band i to contributor
    //                                  i mod R) when R <= FM, else units u with
    //                                  u mod R = c; every contributor stores
    //                                  the units it does not reduce and raises a
    //                                  word per reducer
    //
    // A band reduced by one workgroup is staged and written in one pass; a
    // band split between workgroups goes block by block.
    //
    // One routine serves every role, so the accumulators have a single way out
    // of the registers (separate consumers made the register allocator spill
    // them).  The caller guarantees all waves have left the MAC loop's LDS.
    struct Exit {
        int store_mask, flag_words, fin_mask, fw, lo, hi;
    };
    static constexpr int UNITS = FM * FN;
    // Reducers split bands into blocks only where a wave has few bands (the
    // large tiles' second epilogue form would push their accumulators out of
    // the registers); REDUCERS caps the reducing contributors.
    static constexpr bool kBlockUnits = FM < 4;
    static constexpr int REDUCERS = kBlockUnits ? UNITS : FM;
    static constexpr int EPI_LD = WTN + 8;                     // staged rows: one band wide
    static constexpr int EPI_BYTES = 32 * EPI_LD * 4;
    static constexpr int EPI_PER_STAGE = STAGE / EPI_BYTES;    // waves staging in one LDS stage
    static_assert(EPI_PER_STAGE >= 1 && NW <= EPI_PER_STAGE * NS, "epilogue staging must fit in the stages");
    static_assert(UNITS <= 16 && REDUCERS <= 8, "unit masks and flag words");

    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t peer_slot(const KArgs& ka, int k, bool valid) {
        return __builtin_amdgcn_make_buffer_rsrc(ka.partials + (size_t)uni(k) * SLOT, (short)0,
                                                 valid ? SLOT * 4 : 0, kBufferFlags);
    }

    // Unit (i, j) of peer slot rs into buf (zero-length rs: zeros, no access).
    static __device__ __forceinline__ void load_unit(__amdgpu_buffer_rsrc_t rs, int i, int j, u32x4 (&buf)[CPB],
                                                     int tid) {
#pragma unroll
        for (int r = 0; r < CPB; ++r)
            buf[r] = __builtin_amdgcn_raw_buffer_load_b128(rs, (((i * FN + j) * CPB + r) * THREADS + tid) * 16, 0,
                                                           kCoherent);
    }

    // Adds the copy of peer k (in buf) to the sum of unit (i, j).
    static __device__ __forceinline__ void take_unit(Acc& acc, Blk& T, bool& ahead, int i, int j, int k, int wg,
                                                     const u32x4 (&buf)[CPB]) {
        if (k < wg) {                        // a peer ahead of this workgroup: into the apart sum
#pragma unroll
            for (int r = 0; r < CPB; ++r) blk_take_chunk(T, r, buf[r], !ahead);
            ahead = true;
        } else {
            if (ahead) acc_add_blk(acc, i, j, T);
            ahead = false;
#pragma unroll
            for (int r = 0; r < CPB; ++r) acc_add_chunk(acc, i, j, r, buf[r]);
        }
    }

    static __device__ __forceinline__ int next_peer(int k, int wg) { return k + 1 == wg ? k + 2 : k + 1; }

    static __device__ __forceinline__ void reduce_unit(const KArgs& ka, Acc& acc, int i, int j, int lo, int hi,
                                                       int wg, int tid) {
        Blk T;
        bool ahead = false;
        if constexpr (DT == DT_F64) {
            // One copy at a time, half a block per load (the FP64 tiles trade
            // the pipeline for occupancy and registers).  Each element still
            // takes the peers in the same order.
            constexpr int H = CPB / 2;
            for (int k = lo; k <= hi; ++k) {
                if (k == wg) continue;
                const __amdgpu_buffer_rsrc_t rs = peer_slot(ka, k, true);
                const bool into_apart = k < wg, first = !ahead;
                if (!into_apart && ahead) acc_add_blk(acc, i, j, T);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    u32x4 buf[H];
#pragma unroll
                    for (int r = 0; r < H; ++r)
                        buf[r] = __builtin_amdgcn_raw_buffer_load_b128(
                            rs, (((i * FN + j) * CPB + h * H + r) * THREADS + tid) * 16, 0, kCoherent);
#pragma unroll
                    for (int r = 0; r < H; ++r) {
                        if (into_apart) blk_take_chunk(T, h * H + r, buf[r], first);
                        else acc_add_chunk(acc, i, j, h * H + r, buf[r]);
                    }
                }
                ahead = into_apart;
            }
            if (ahead) acc_add_blk(acc, i, j, T);
            return;
        }
        u32x4 buf0[CPB], buf1[CPB];
        int k = lo == wg ? lo + 1 : lo;
        load_unit(peer_slot(ka, k, k <= hi), i, j, buf0, tid);
        while (k <= hi) {
            int k1 = next_peer(k, wg);
            load_unit(peer_slot(ka, k1, k1 <= hi), i, j, buf1, tid);
            take_unit(acc, T, ahead, i, j, k, wg, buf0);
            __builtin_amdgcn_sched_barrier(0);
            if (k1 > hi) break;
            const int k2 = next_peer(k1, wg);
            load_unit(peer_slot(ka, k2, k2 <= hi), i, j, buf0, tid);
            take_unit(acc, T, ahead, i, j, k1, wg, buf1);
            __builtin_amdgcn_sched_barrier(0);
            k = k2;
        }
        if (ahead) acc_add_blk(acc, i, j, T);   // the peers ahead were the last ones
    }

    // Segment timestamps of a timed run (one lane writes them; ts is null otherwise).
    static __device__ __forceinline__ void stamp(uint64_t* ts, int f, int tid) {
        if (ts && tid == 0) ts[f] = __builtin_amdgcn_s_memrealtime();
    }
    // The shader-clock counter, into field f of a timed run's record.
    static __device__ __forceinline__ void stamp_clock(uint64_t* ts, int f, int tid) {
        if (ts && tid == 0) ts[f] = __builtin_amdgcn_s_memtime();
    }

    static __device__ __forceinline__ void finish(const KArgs& ka, const Prob& a, int tile, Acc& acc, int tid,
                                                  const Stages& sts, int wg, const Exit& x, uint64_t* ts) {
        tid = opaque(tid);
        const int lane = tid & 63, w = tid >> 6, wm = w / WN, wn = w % WN;
        const int g = lane >> 5, l32 = lane & 31;
        const int store_mask = uni(x.store_mask), fin_mask = uni(x.fin_mask);
        if (store_mask) {
            const __amdgpu_buffer_rsrc_t own = slot_rsrc(ka.partials + (size_t)wg * SLOT);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    if ((store_mask >> (i * FN + j)) & 1) {
#pragma unroll
                        for (int r = 0; r < CPB; ++r) {
                            const int q = (i * FN + j) * CPB + r;
                            __builtin_amdgcn_raw_buffer_store_b128(acc_chunk(acc, i, j, r), own,
                                                                   (q * THREADS + tid) * 16, 0, kCoherent);
                        }
                    }
            wait_vmem();          // this wave's coherent partial stores have completed
            __syncthreads();      // ... and so have every other wave's
            if (tid == 0) {
                int32_t* f = ka.flags + (size_t)wg * kFlagStrideInts;
                for (int b = 0; b < 8; ++b)
                    if ((x.flag_words >> b) & 1) __hip_atomic_store(f + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        stamp(ts, 2, tid);
        if (!fin_mask) {
            stamp(ts, 3, tid);
            return;
        }
        const int fw = uni(x.fw), lo = uni(x.lo), hi = uni(x.hi);
        // every wave polls the flags itself (wave-uniform loops: no divergent
        // region around the accumulators)
        wait_flags(ka.flags + fw, lo, min(hi, wg - 1), ka.spin_limit, ka.err);
        wait_flags(ka.flags + fw, max(lo, wg + 1), hi, ka.spin_limit, ka.err);
        stamp(ts, 3, tid);
        int m0, n0;
        tile_origin(a, tile, m0, n0);
        m0 += wm * WTM;
        n0 += wn * WTN;
        const int sj = w / EPI_PER_STAGE;
        unsigned char* base = sts.template at<0>();
        if (sj == 1) base = sts.template at<1 % NS>();
        if constexpr (NS > 2) if (sj == 2) base = sts.template at<2 % NS>();
        if constexpr (NS > 3) if (sj == 3) base = sts.template at<3 % NS>();
        if constexpr (NS > 4) if (sj == 4) base = sts.template at<4 % NS>();
        float* st = reinterpret_cast<float*>(base + (w % EPI_PER_STAGE) * EPI_BYTES);
        float sc = a.alpha;
        if (ka.scale_a) sc *= *ka.scale_a;
        if (ka.scale_b) sc *= *ka.scale_b;
        const bool peers = hi >= lo && !(lo == wg && hi == wg);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            constexpr int BAND = (1 << FN) - 1;
            const bool whole = ((fin_mask >> (i * FN)) & BAND) == BAND;
            if constexpr (DT == DT_F64) {
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (!((fin_mask >> (i * FN + j)) & 1)) continue;
                    if (peers) reduce_unit(ka, acc, i, j, lo, hi, wg, tid);
                    write_block_f64(a, double(sc), acc, i, j, m0, n0, lane);
                }
            } else if (whole) {
                // the whole band: reduce its blocks, stage them side by side, one write pass
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (peers) reduce_unit(ka, acc, i, j, lo, hi, wg, tid);
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        st[(8 * (r >> 2) + 4 * g + (r & 3)) * EPI_LD + j * 32 + l32] = acc.v[i][j][r];
                }
                constexpr int LPR = WTN / 8;
                const int col = n0 + (lane % LPR) * 8;
                const int ncol = min(max(a.N - col, 0), 8);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (ka.out_dtype == DT_F32) write_band<DT_F32, WTN>(a, sc, st, m0 + i * 32, col, ncol, lane);
                else if (ka.out_dtype == DT_BF16) write_band<DT_BF16, WTN>(a, sc, st, m0 + i * 32, col, ncol, lane);
                else write_band<DT_F16, WTN>(a, sc, st, m0 + i * 32, col, ncol, lane);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else if constexpr (kBlockUnits) {
                // single blocks of the band
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if (!((fin_mask >> (i * FN + j)) & 1)) continue;
                    if (peers) reduce_unit(ka, acc, i, j, lo, hi, wg, tid);
                    const int col = n0 + j * 32 + (lane % 4) * 8;
                    const int ncol = min(max(a.N - col, 0), 8);
#pragma unroll
                    for (int r = 0; r < 16; ++r) st[(8 * (r >> 2) + 4 * g + (r & 3)) * EPI_LD + l32] = acc.v[i][j][r];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (ka.out_dtype == DT_F32) write_band<DT_F32, 32>(a, sc, st, m0 + i * 32, col, ncol, lane);
                    else if (ka.out_dtype == DT_BF16) write_band<DT_BF16, 32>(a, sc, st, m0 + i * 32, col, ncol, lane);
                    else write_band<DT_F16, 32>(a, sc, st, m0 + i * 32, col, ncol, lane);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
        }
        if (peers) {
            __syncthreads();      // every wave has seen every flag: clear the words waited on
            if (tid == 0)
                for (int k = lo; k <= hi; ++k)
                    if (k != wg)
                        __hip_atomic_store(ka.flags + (size_t)k * kFlagStrideInts + fw, 0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // Grouped launches: the problem holding a global iteration / tile (the
    // last entry whose base is <= x; empty problems share the next base and
    // are skipped by taking the last).
    static __device__ __forceinline__ int find_iter(const KArgs& a, int64_t x) {
        int lo = 0, hi = a.G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.group[mid].iter_base <= x) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }

    static __device__ __forceinline__ int find_tile(const KArgs& a, int x) {
        int lo = 0, hi = a.G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.group[mid].tile_base <= x) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }

    // Strided batch: the problem holding global tile x (operands offset by
    // its index times the strides); returns the tile's index within it.
    static __device__ __forceinline__ int batch_tile(const KArgs& a, int x, Prob& pr) {
        const int pi = x / a.t1;
        pr.A = reinterpret_cast<const unsigned char*>(pr.A) + int64_t(pi) * a.stride_a;
        pr.B = reinterpret_cast<const unsigned char*>(pr.B) + int64_t(pi) * a.stride_b;
        pr.C = reinterpret_cast<unsigned char*>(pr.C) + int64_t(pi) * a.stride_c;
        return x - pi * a.t1;
    }

    static __device__ __forceinline__ Prob entry_prob(const GroupEntry& e, int raster) {
        return Prob{e.A, e.B, e.C, e.lda, e.ldb, e.ldc, e.M, e.N, e.K, e.tn, e.ipt, e.alpha, e.beta, raster, ConvArgs{}};
    }

    // Logical workgroup index of hardware workgroup b.  Workgroups are handed
    // to the XCDs round-robin (b mod xcds), and each XCD has its own L2; the
    // permutation gives every XCD a contiguous range of logical indices, so
    // the Stream-K shares and data-parallel tiles it runs are neighbours.
    // A bijection of [0, grid); xcds = 1 is the identity.
    static __device__ __forceinline__ int logical_wg(int b, int grid, int xcds) {
        if (xcds <= 1) return b;
        const int q = grid / xcds, r = grid % xcds;
        const int x = b % xcds, pos = b / xcds;
        return x < r ? x * (q + 1) + pos : r * (q + 1) + (x - r) * q + pos;
    }

    // Relaxed agent-scope polling of the ready flags of peers first..last,
    // in order, in one loop: coherent loads with no cache invalidation per
    // poll.  All lanes load the same word, so the value is wave-uniform and
    // the loop runs as scalar branches.  Bounded: past spin_limit polls the
    // error word is set and the wait ends.
    static __device__ __forceinline__ void wait_flags(const int32_t* flags, int first, int last, int spin_limit,
                                                      int32_t* err) {
        int spins = 0, peer = first;
        while (peer <= last) {
            if (uni(__hip_atomic_load(flags + (size_t)peer * kFlagStrideInts, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT)) != 0) {
                ++peer;
                continue;
            }
            __builtin_amdgcn_s_sleep(2);
            if (++spins > spin_limit) {
                __hip_atomic_store(err, kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        // Compiler barrier: the partial loads that follow stay after the
        // polls (the hardware issues them only once the loop has seen every
        // flag, as the loop's exit depends on the loaded values).
        asm volatile("" ::: "memory");
    }

    // Even share of the Stream-K iterations: proportional (workgroup x starts
    // at floor(x * T / g)) or leading (the first T mod g workgroups get q + 1).
    static __device__ __forceinline__ int share_start(const KArgs& a, int x) {
        if (a.sk_prop) return int(int64_t(x) * a.sk_iters / a.g_sk);
        return x * a.sk_q + min(x, a.sk_r);
    }

    // The workgroup whose share holds iteration i.
    static __device__ __forceinline__ int owner_of(const KArgs& a, int i) {
        if (a.sk_prop) return int((int64_t(i + 1) * a.g_sk - 1) / a.sk_iters);
        const int q = a.sk_q, r = a.sk_r;
        return (i < r * (q + 1)) ? i / (q + 1) : r + (i - r * (q + 1)) / q;
    }

    // The segment walk of the basic Stream-K algorithm (with the hybrids'
    // data-parallel tiles): a workgroup takes its contiguous share of the
    // Stream-K iterations, cut at tile seams, before or after its whole
    // data-parallel tiles.  Iterations and tiles are global indices; a grouped
    // launch concatenates the problems' iteration spaces.  FULL = false is the
    // lean form for one plain GEMM (no group table, no batch, no trace or
    // timestamps): without their values live across the loop, the segment
    // walk and epilogue spill fewer scalars (the full form runs plain GEMMs
    // 2.3 % slower over the BF16 shape sweep).  Its problem fields pass
    // through opaque_prob each segment, as the full form's may change.
    template <bool FULL>
    static __device__ __forceinline__ void run(const KArgs& a, const Stages& st) {
        const int tid = threadIdx.x;
        const int wg = logical_wg(blockIdx.x, a.grid, a.xcds);
        int sk_it = 0, sk_end = 0;
        if (wg < a.g_sk) {
            sk_it = share_start(a, wg);
            sk_end = share_start(a, wg + 1);
        }
        int dp_tile = a.sk_tiles + wg;
        int seq = 0;
        const Prob single = {a.A, a.B, a.C, a.lda, a.ldb, a.ldc, a.M, a.N, a.K, a.tn, a.ipt, a.alpha, a.beta,
                             a.raster, a.conv};
        Acc acc;
        for (;;) {
            const bool sk_left = sk_it < sk_end, dp_left = dp_tile < a.t;
            if (!sk_left && !dp_left) break;
            const bool take_sk = a.sk_first ? sk_left : !dp_left;
            Prob pr = single;
            int gtile, tile, lo, hi, role, peer_end = -1;
            if (take_sk) {
                int first;
                if (FULL && a.G) {
                    const GroupEntry& e = a.group[find_iter(a, sk_it)];
                    pr = entry_prob(e, a.raster);
                    tile = int((sk_it - e.iter_base) / e.ipt);
                    first = int(e.iter_base) + tile * e.ipt;
                    gtile = e.tile_base + tile;
                } else {
                    tile = sk_it / a.ipt;
                    first = tile * a.ipt;
                    gtile = tile;
                    if (FULL && a.batch > 1) tile = batch_tile(a, tile, pr);
                }
                const int last = first + pr.ipt;
                lo = sk_it - first;
                hi = min(sk_end, last) - first;
                if (sk_it != first) {
                    role = ROLE_PARTIAL;
                } else if (sk_end < last) {
                    role = ROLE_OWNER;
                    peer_end = owner_of(a, last - 1);
                } else {
                    role = ROLE_FULL;
                }
                sk_it = last;
            } else {
                gtile = dp_tile;
                tile = dp_tile;
                if (FULL && a.G) {
                    const GroupEntry& e = a.group[find_tile(a, dp_tile)];
                    pr = entry_prob(e, a.raster);
                    tile = dp_tile - e.tile_base;
                } else if (FULL && a.batch > 1) {
                    tile = batch_tile(a, dp_tile, pr);
                }
                lo = 0;
                hi = pr.ipt;
                role = ROLE_FULL;
                dp_tile += a.grid;
            }
            pr = FULL ? uniform(pr) : opaque_prob(pr);
            tile = uni(tile);
            lo = uni(lo);
            hi = uni(hi);
            if (FULL && a.trace && tid == 0 && seq < a.trace_per_wg) {
                int32_t* rec = a.trace + ((size_t)wg * a.trace_per_wg + seq) * kTraceFields;
                rec[0] = wg; rec[1] = seq; rec[2] = gtile; rec[3] = lo; rec[4] = hi; rec[5] = role;
                rec[6] = role == ROLE_OWNER ? wg + 1 : -1;
                rec[7] = role == ROLE_OWNER ? peer_end : -1;
            }
            uint64_t* ts = FULL && a.times && seq < a.trace_per_wg
                               ? a.times + ((size_t)wg * a.trace_per_wg + seq) * kTimeFields
                               : nullptr;
            ++seq;
            stamp(ts, 0, tid);
            stamp_clock(ts, 5, tid);

            mac_loop(pr, st, tile, lo, hi, acc, tid);
            stamp(ts, 1, tid);

            constexpr int ALL = (1 << UNITS) - 1;
            Exit x = {0, 0, ALL, 0, 1, 0};            // whole tile: write every unit
            if (take_sk && a.coop_s) {
                // split fix-up: the plan cut every Stream-K tile into coop_s
                // shares, one per workgroup; wg is contributor wg mod coop_s,
                // and the first R contributors reduce (whole bands if R <= FM)
                const int c = wg % a.coop_s, first = wg - c;
                const int R = min(a.coop_s, REDUCERS);
                int mine = 0;
                if (c < R)
                    for (int u = 0; u < UNITS; ++u)
                        if ((R <= FM ? (u / FN) % R : u % R) == c) mine |= 1 << u;
                x.store_mask = ALL & ~mine;
                x.flag_words = ((1 << R) - 1) & ~(c < R ? 1 << c : 0);
                x.fin_mask = mine;
                x.fw = c;
                x.lo = first;
                x.hi = first + a.coop_s - 1;
            } else if (role == ROLE_PARTIAL) {
                x = Exit{ALL, 1, 0, 0, 1, 0};
            } else if (role == ROLE_OWNER) {
                x = Exit{0, 0, ALL, 0, wg + 1, peer_end};
            }
            finish(a, pr, tile, acc, tid, st, wg, x, ts);
            stamp(ts, 4, tid);
            stamp_clock(ts, 6, tid);
        }
    }
};

// FULL: the instantiation for launches with a group table, a batch, a trace
// or timestamps; plain GEMMs launch the lean one.
template <int DT, bool AKC, bool BKC, int V, bool FULL>
__global__ void __launch_bounds__((kThreadsOf<DT, V>)) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<DT, V>)))
skgemm_kernel(KArgs a) {
    using G = Gemm<DT, AKC, BKC, V>;
    constexpr int S = G::STAGE;
    __shared__ __attribute__((aligned(1024))) unsigned char st0[S];
    __shared__ __attribute__((aligned(1024))) unsigned char st1[S];
    typename G::Stages sts{st0, st1, nullptr, nullptr, nullptr};
    if constexpr (G::NS == 2) {
        G::template run<FULL>(a, sts);
    } else if constexpr (G::NS == 3) {
        __shared__ __attribute__((aligned(1024))) unsigned char st2[S];
        sts.s2 = st2;
        G::template run<FULL>(a, sts);
    } else if constexpr (G::NS == 4) {
        __shared__ __attribute__((aligned(1024))) unsigned char st2[S];
        __shared__ __attribute__((aligned(1024))) unsigned char st3[S];
        sts.s2 = st2;
        sts.s3 = st3;
        G::template run<FULL>(a, sts);
    } else {
        static_assert(G::NS == 5, "2 to 5 pipeline stages");
        __shared__ __attribute__((aligned(1024))) unsigned char st2[S];
        __shared__ __attribute__((aligned(1024))) unsigned char st3[S];
        __shared__ __attribute__((aligned(1024))) unsigned char st4[S];
        sts.s2 = st2;
        sts.s3 = st3;
        sts.s4 = st4;
        G::template run<FULL>(a, sts);
    }
}

}  // namespace skg
