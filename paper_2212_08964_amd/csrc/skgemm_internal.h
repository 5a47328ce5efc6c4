// Internal declarations shared by the library's planner, ABI layer and kernels.
#pragma once

#include <stdint.h>
#include <stddef.h>

namespace skg {

enum DType : int32_t { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2, DT_F8 = 3, DT_F64 = 4 };
constexpr int kDTypes = 5;                 // number of DType values
enum Role : int32_t { ROLE_FULL = 0, ROLE_PARTIAL = 1, ROLE_OWNER = 2 };

constexpr int kFlagStrideInts = 32;        // one 128-byte line per ready flag
constexpr size_t kWsHeaderBytes = 256;     // error word lives at offset 0
// The flag area has a fixed place and size (ahead of the partial tiles), so a
// workspace can serve plans with different grids one after another: a
// plan's partial tiles never overlap another plan's flags.
constexpr int kMaxFlagLines = 4096;        // Stream-K workgroups a plan may have
// The automatic policy stays data-parallel from this many full waves on.
constexpr int kAutoMaxWaves = 4;
constexpr int kTraceFields = 8;
// Timestamps per traced segment (device real-time clock): start, MAC loop
// done, partial stores and flags done, fix-up waits done, segment done.
constexpr int kTimeFields = 7;
constexpr int32_t kErrTimeout = 6;

// Compiled tile configurations per input type (BM x BN x BK).
// Tile (bm x bn, k-slab bk) and LDS pipeline stages per input type / variant.
struct TileCfg { int bm, bn, bk, ns; };
constexpr TileCfg kTileF32 = {128, 128, 32, 2};
constexpr TileCfg kTile16 = {256, 256, 64, 2};    // bf16 and f16
constexpr TileCfg kTile16S = {128, 128, 64, 2};   // bf16 and f16, small-tile variant
constexpr TileCfg kTile16K = {64, 256, 64, 2};    // bf16 and f16, skinny-M variant (M <= 64)
constexpr TileCfg kTile16T = {256, 64, 64, 2};    // bf16 and f16, skinny-N variant (N <= 64)
constexpr TileCfg kTileF8 = {256, 256, 128, 2};
constexpr TileCfg kTileF8S = {128, 128, 128, 2};   // fp8, small-tile variant
constexpr TileCfg kTileF64 = {64, 64, 16, 2};
constexpr TileCfg kTileF64L = {128, 128, 16, 2};   // fp64, large-tile variant
constexpr TileCfg kTile16D = {128, 128, 64, 3};   // bf16 and f16, small tile on three LDS stages

// One problem of a grouped launch (device table entry, 128 bytes).  Shapes are
// as launched (operands already swapped when C is column-major).
struct GroupEntry {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    int64_t iter_base;          // global MAC-loop iteration of the problem's first tile
    int32_t M, N, K, tm, tn, ipt;
    int32_t tile_base;          // global index of the problem's first tile
    float alpha, beta;
    int32_t pad[9];
};
static_assert(sizeof(GroupEntry) == 128, "group table entry layout");

// Implicit-GEMM convolution (the GEMM view of a 2-D convolution): input x
// NHWC, filters KRSC, output NPQK.  GEMM rows m = (n P + p) Q + q, columns =
// output channels, reduction kk = (r S + s) C + c; A[m][kk] is gathered from
// x (zero outside the image), B is the filters as a column-major matrix with
// leading dimension R S C, C the output as a row-major matrix.
struct ConvArgs {
    int32_t n, h, w, c;                 // input
    int32_t p, q, r, s;                 // output size and filter window
    int32_t pad_h, pad_w, str_h, str_w, dil_h, dil_w;
};

// Kernel arguments, passed by value.  Operands are described relative to the
// reduction: an operand is "K-contiguous" when consecutive k are adjacent in
// memory (row-major A, column-major B).
struct KArgs {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t tm, tn, t, ipt;
    int32_t sk_tiles, g_sk, sk_iters, sk_q, sk_r, grid;
    int32_t sk_first, dp_only;
    float alpha, beta;
    const float* scale_a;
    const float* scale_b;
    int32_t out_dtype;
    int32_t vec_a, vec_b;      // bytes per vector global load: 16, 8, 4, 2 or 1
    float* partials;
    int32_t* flags;
    int32_t* err;
    int32_t* trace;
    uint64_t* times;           // kTimeFields per trace record, or null
    int32_t trace_per_wg;
    int32_t spin_limit;
    const GroupEntry* group;   // grouped launch: G problem entries (else null)
    int32_t G;
    int32_t sk_prop;           // proportional even share (else leading: first sk_r get sk_q + 1)
    int32_t raster;            // tile rows per raster group (1 = row-major)
    int32_t xcds;              // XCDs the workgroups are spread over (1 = no remapping)
    int32_t coop_s;            // >= 2: every Stream-K tile has coop_s one-segment shares and the
                               // split fix-up reduces it (0 = owner fix-up)
    // Strided batch of equal problems (batch > 1): tile index x is tile
    // x mod t1 of problem x / t1, whose operands start stride_* bytes after
    // the previous problem's.
    int32_t batch, t1;
    int64_t stride_a, stride_b, stride_c;
    ConvArgs conv;             // implicit-GEMM convolution kernels only
};

// Tile variants: 0 = the type's default tile, 1 = the small 16-bit / FP8 tile
// (four waves) or the large FP64 tile, 2 = the small 16-bit tile on eight
// waves.
// 3 and 4: the 256x256 and the four-wave 128x128 16-bit tiles with the
// implicit-GEMM convolution gather for A.  5: the skinny 64x256 16-bit tile
// (four waves side by side) for problems of at most 64 rows; 6: the 256x64
// tile (four waves stacked) for problems of at most 64 columns, and 7 the
// same with the convolution gather (at most 64 output channels).  8: the
// eight-wave 128x128 16-bit tile on three LDS stages (two slabs in flight),
// one workgroup per CU; the planner substitutes it for variants 1 and 2
// where the grid fits one workgroup per CU, never as a candidate of its own.
// 9: the same with the convolution gather, substituted for variant 4.
constexpr int kVariants = 10;
constexpr int kVariantDeep = 8;
constexpr int kVariantDeepConv = 9;
constexpr bool is_conv_variant(int v) { return v == 3 || v == 4 || v == 7 || v == 9; }

// Copy `lines` lines of `cols` elements of eb bytes (line i at src + i * ld)
// to dst with leading dimension ldd, on stream.  Returns a hipError_t value.
int launch_pack(const void* src, int64_t ld, int64_t lines, int64_t cols, void* dst, int64_t ldd, int eb,
                void* stream);

// Launch one Stream-K GEMM kernel.  Returns a hipError_t value.
int launch_gemm(int dtype, bool a_kcontig, bool b_kcontig, int variant, const KArgs& args, int grid,
                void* stream);
// Workgroups of the kernel that fit on one CU at once (0 on failure).
int kernel_occupancy(int dtype, bool a_kcontig, bool b_kcontig, int variant);
bool kernel_exists(int dtype, bool a_kcontig, bool b_kcontig, int variant);
// Threads per workgroup of the kernel.
int kernel_threads(int dtype, int variant);

// Per-tensor E4M3 quantisation (three launches on `stream`).
int launch_quantize(int dtype, const void* x, int64_t rows, int64_t cols, int64_t ldx, bool x_col, uint8_t* q,
                    int64_t ldq, bool q_col, float* scale, float* partial, void* stream);
// FP32 scratch values the quantiser needs.
int quant_workspace_floats();

}  // namespace skg
