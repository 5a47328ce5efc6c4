/*
 * skgemm: Stream-K GEMM for AMD Instinct MI355X (gfx950).
 *
 * Computes C = alpha * (s_A * s_B) * A * B + beta * C, the GEMM problem of the
 * Background section of "Stream-K: Work-centric Parallel Decomposition for
 * Dense Matrix-Matrix Multiplication on the GPU" (dissertation chapter of
 * arXiv 2212.08964), with the work split by MAC-loop iteration across a grid
 * of persistent workgroups as in the basic Stream-K algorithm and its
 * data-parallel hybrids (Data-parallel Hybridization subsection).
 *
 * Conventions shared by every entry point:
 *  - Shapes: A is M x K, B is K x N, C is M x N.  Each operand is row- or
 *    column-major with its own leading dimension (elements, not bytes).
 *  - Element types: A and B share one input type; C is FP32, BF16 or FP16
 *    (FP8 inputs write FP32, BF16 or FP16).  Accumulation and the fix-up of
 *    partial tiles are FP32.  Output rounding is round-to-nearest-even.
 *  - Device pointers: A, B, C, scales, workspace, trace and descriptor arrays
 *    are device memory owned by the caller.  The library owns only plans.
 *  - Streams: runs are asynchronous on the given hipStream_t (NULL = default
 *    stream).  Plans are immutable after creation and may be shared by
 *    threads; a workspace must not be used by two runs in flight at once.
 *  - Errors: every call returns a status and never throws.  Argument errors
 *    are reported before anything is launched.  beta == 0 never reads C.
 *    K == 0 gives C = beta * C; M == 0 or N == 0 launches nothing.
 */
#ifndef SKGEMM_H
#define SKGEMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SKGEMM_OK = 0,
    SKGEMM_ERR_INVALID_ARG = 1,   /* bad shape, leading dimension, pointer or enum */
    SKGEMM_ERR_UNSUPPORTED = 2,   /* valid request the library does not implement */
    SKGEMM_ERR_WORKSPACE = 3,     /* workspace missing, misaligned or too small */
    SKGEMM_ERR_CAPACITY = 4,      /* grid larger than the co-resident workgroups
                                     (or than 4096 Stream-K workgroups) */
    SKGEMM_ERR_HIP = 5,           /* a HIP runtime call failed */
    SKGEMM_ERR_TIMEOUT = 6        /* a bounded fix-up wait expired on the device */
} skgemm_status_t;

typedef enum { SKGEMM_ROW_MAJOR = 0, SKGEMM_COL_MAJOR = 1 } skgemm_layout_t;

typedef enum {
    SKGEMM_F32 = 0,
    SKGEMM_F16 = 1,
    SKGEMM_BF16 = 2,
    SKGEMM_F8E4M3 = 3,            /* OCP E4M3FN, used with per-tensor scales */
    SKGEMM_F64 = 4                /* FP64 in, FP64 accumulate, fix-up and out */
} skgemm_dtype_t;

/* Work decomposition (Work Decomposition Strategies section and
 * Data-parallel Hybridization subsection). */
typedef enum {
    SKGEMM_POLICY_AUTO = 0,       /* this library's rule for MI355X (not the paper's):
                                     DP when the tiles fill whole waves or make four
                                     full waves or more; otherwise the remainder
                                     tiles (all tiles when there are fewer than
                                     workgroups) are split into s equal parts each,
                                     s from the grid-size model over 1 .. p / tiles
                                     (with the occupancy term of
                                     skgemm_model_constants): s = 1 is DP, else
                                     basic SK (no full wave) or DP + one-tile SK
                                     with g = s * tiles.  A grouped plan whose
                                     problems differ in iterations per tile takes
                                     SKGEMM_POLICY_PAPER's choice. */
    SKGEMM_POLICY_DP = 1,         /* one workgroup per output tile */
    SKGEMM_POLICY_SK = 2,         /* basic Stream-K over all tiles */
    SKGEMM_POLICY_DP_1TILE_SK = 3,/* full DP waves, Stream-K over the remainder tiles */
    SKGEMM_POLICY_2TILE_SK_DP = 4,/* Stream-K over remainder + one wave, then DP waves */
    SKGEMM_POLICY_PAPER = 5       /* the paper's own selection (Data-parallel
                                     Hybridization subsection): DP when the tiles
                                     fill whole waves; basic SK with g from the
                                     grid-size model over [tiles, p] when there are
                                     fewer tiles than workgroups; two-tile SK + DP
                                     from hybrid_min_waves full waves on; DP +
                                     one-tile SK otherwise */
} skgemm_policy_t;

typedef struct {
    skgemm_policy_t policy;       /* default SKGEMM_POLICY_AUTO */
    int32_t force_g;              /* >0: Stream-K grid size instead of the model's choice */
    int32_t tile_m, tile_n, tile_k;   /* 0 = the planner picks among the dtype's
                                         compiled tiles by modelled time; else must
                                         name one: FP32 128x128x32; FP16/BF16
                                         256x256x64, 128x128x64, 64x256x64 (A
                                         K-contiguous; picked automatically only
                                         where every launched problem has at most
                                         64 rows) or 256x64x64 (B K-contiguous; at
                                         most 64 columns); FP8 256x256x128 or
                                         128x128x128; FP64 64x64x16 or 128x128x16.
                                         A named tile with no kernel for the
                                         operands' contiguity: SKGEMM_ERR_UNSUPPORTED.
                                         A 16-bit 128x128x64 plan (GEMM or
                                         convolution) whose grid is at most the
                                         CU count runs an eight-wave kernel with
                                         three LDS stages (one workgroup per CU;
                                         plan_info field 29) unless tile_waves
                                         asks for four */
    int32_t hybrid_min_waves;     /* full waves needed for the two-tile hybrid (default 2) */
    int32_t num_cus;              /* >0: plan for this many CUs instead of querying */
    int32_t occupancy;            /* >0: workgroups per CU instead of querying */
    int32_t raster_rows;          /* output tiles are numbered down groups of this many
                                     tile rows, column by column (0 = default 8,
                                     1 = row-major); does not change the schedule
                                     over tile indices, only which block a tile is */
    int32_t xcds;                 /* hardware workgroup b runs as logical workgroup
                                     perm(b) so that each of this many XCDs (the GPU
                                     hands workgroups to XCDs round-robin) gets a
                                     contiguous range of logical workgroups
                                     (0 = default 8, 1 = identity); the schedule over
                                     logical workgroups is unchanged */
    int32_t share;                /* even share of the Stream-K iterations (each
                                     workgroup gets floor(T/g) or ceil(T/g)):
                                     SKGEMM_SHARE_PROPORTIONAL (default) starts
                                     workgroup x at floor(x*T/g), so when g is a
                                     multiple s of the Stream-K tile count every tile
                                     is cut into s parts at the same k-offsets;
                                     SKGEMM_SHARE_LEADING gives the T mod g extra
                                     iterations to the first workgroups */
    int32_t fixup;                /* SKGEMM_FIXUP_AUTO (default): when every Stream-K
                                     tile is cut into s >= 2 shares that start and
                                     end on the tile (one GEMM, g = s * tiles, and s
                                     at most the iterations per tile with the
                                     proportional share, a divisor of them with the
                                     leading share), the first
                                     two workgroups of a tile each reduce and write
                                     half of its 32-row bands and every other share
                                     is stored for them; otherwise, and always with
                                     SKGEMM_FIXUP_OWNER, the workgroup holding the
                                     tile's first iteration reduces and writes the
                                     whole tile (the paper's fix-up).  Both add the
                                     shares in the same order: the results are
                                     bitwise identical. */
    int32_t tile_waves;           /* 0 = any; else the wavefronts per workgroup of the
                                     tile configuration (the 128x128x64 16-bit tile
                                     exists on 4 and on 8 waves) */
    int32_t spin_limit;           /* 0 = default (2^22): polls of a peer's ready flag
                                     (a short sleep between polls) after which a
                                     fix-up wait gives up: it sets the workspace's
                                     error word (SKGEMM_ERR_TIMEOUT from
                                     skgemm_check_device_error) and the workgroup
                                     finishes with the sum it has, so the kernel
                                     always exits.  A small value forces that path
                                     (tests of the error handling). */
    int32_t relayout;             /* copy of misaligned operands into 128-byte
                                     aligned lines before the GEMM (single-GEMM
                                     plans, see skgemm_run): 0 = where it is
                                     predicted to pay (the operand is read once
                                     per panel of the other operand: the
                                     misaligned bytes moved, its size times that
                                     panel count, against the copy's 2 bytes
                                     moved per operand byte), -1 = never,
                                     1 / 2 / 3 = always
                                     for A / B / both (the operands as given by
                                     the caller) when their lines are misaligned */
} skgemm_options_t;

typedef enum { SKGEMM_SHARE_PROPORTIONAL = 0, SKGEMM_SHARE_LEADING = 1 } skgemm_share_t;
typedef enum { SKGEMM_FIXUP_AUTO = 0, SKGEMM_FIXUP_OWNER = 1 } skgemm_fixup_t;

/* Fills *opt with the defaults. */
void skgemm_default_options(skgemm_options_t* opt);

typedef struct skgemm_plan_s* skgemm_plan_t;

/* Plan one GEMM (host arithmetic only; queries device 0's properties unless
 * opt->num_cus and opt->occupancy are set).  la / lb / lc are the layouts of
 * A, B and C; ta == tb is required.  FP8 needs A row-major and B
 * column-major (K contiguous in both); skgemm_quantize_e4m3 writes either.
 * On success *out receives a plan that skgemm_plan_destroy frees.  With
 * SKGEMM_LOG=1 in the environment every plan function prints one line per
 * plan it builds on stderr (launch kind, shape, tile, resolved policy and
 * grid, modelled time). */
skgemm_status_t skgemm_plan(skgemm_plan_t* out, int64_t M, int64_t N, int64_t K,
                            skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc,
                            skgemm_dtype_t ta, skgemm_dtype_t tb, skgemm_dtype_t tc,
                            const skgemm_options_t* opt);

/* Bytes of device workspace a run of this plan needs (0 when the plan has no
 * Stream-K region and re-lays out no operand).  The workspace holds an error
 * word, the ready flags (a fixed area of 512 KiB for up to 4096 Stream-K
 * workgroups) and the FP32 partial tiles, one per Stream-K workgroup (the
 * fix-up part, plan_info field 28), then, for a single-GEMM plan that the
 * model says gains from it, room for a copy of A and/or B with 128-byte
 * aligned lines (plan_info fields 26 and 27; see skgemm_run).  It must be
 * 256-byte aligned and zero-filled once after allocation; the kernel leaves
 * its flags at zero again on success, so it can be reused without clearing,
 * also by other plans (the flag area is at the same place for every plan).
 * After SKGEMM_ERR_TIMEOUT it must be zero-filled again. */
skgemm_status_t skgemm_workspace_size(skgemm_plan_t plan, size_t* bytes);

/* Run a planned GEMM.  lda/ldb/ldc follow each operand's layout and must be
 * at least its contiguous extent.  scale_a / scale_b point to one FP32 value
 * on the device each (NULL = 1).  workspace may be NULL when the workspace
 * size is 0.  When the plan re-lays out an operand and its leading dimension
 * in bytes is not a multiple of 128, the run first copies it into the
 * workspace with 128-byte aligned lines (a second kernel on the same stream)
 * and multiplies the copy: the result is bitwise the same.  With a workspace
 * smaller than skgemm_workspace_size but at least its fix-up part the run
 * multiplies the operands as given. */
skgemm_status_t skgemm_run(skgemm_plan_t plan,
                           const void* A, int64_t lda, const void* B, int64_t ldb,
                           void* C, int64_t ldc, float alpha, float beta,
                           const float* scale_a, const float* scale_b,
                           void* workspace, size_t ws_bytes, hipStream_t stream);

/* skgemm_run for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc): the fix-up
 * workspace is a 64 MiB device array the library holds on every GPU it runs
 * on until the process ends, so the caller passes no workspace.  Plans whose
 * fix-up workspace (plan_info field 28) exceeds 64 MiB are refused with
 * SKGEMM_ERR_WORKSPACE (e.g. more than 254 Stream-K workgroups with
 * 256x256 FP32 partial tiles); operands are multiplied as given (no
 * re-layout copy).  Allocates nothing: before the GEMM it
 * clears the error word and the plan's flag lines with a small kernel on
 * `stream` (capturable), then runs skgemm_run on the array.  All calls on
 * one GPU share its array: calls that overlap in time on one GPU (on
 * different streams) race and give wrong results; a fix-up timeout of one
 * call is not reported (the next call clears the error word). */
skgemm_status_t skgemm_run_noalloc(skgemm_plan_t plan,
                                   const void* A, int64_t lda, const void* B, int64_t ldb,
                                   void* C, int64_t ldc, float alpha, float beta,
                                   const float* scale_a, const float* scale_b, hipStream_t stream);

/* Number of schedule records a traced run of this plan can write: the number
 * of launched workgroups times the most segments any of them performs. */
skgemm_status_t skgemm_trace_capacity(skgemm_plan_t plan, size_t* n_records);

/* Same as skgemm_run, and each workgroup also writes one record of 8 int32
 * per segment it performs, in execution order, into trace (device memory of
 * at least skgemm_trace_capacity records; unused records are untouched):
 *   {workgroup, sequence number, tile, first k-iteration, end k-iteration,
 *    role (0 full, 1 partial, 2 owner), first peer, last peer (-1 if none)}.
 * Record (wg, seq) is at index wg * (capacity / grid) + seq. */
skgemm_status_t skgemm_run_traced(skgemm_plan_t plan,
                                  const void* A, int64_t lda, const void* B, int64_t ldb,
                                  void* C, int64_t ldc, float alpha, float beta,
                                  const float* scale_a, const float* scale_b,
                                  void* workspace, size_t ws_bytes,
                                  int32_t* trace, size_t trace_records, hipStream_t stream);

/* Same as skgemm_run_traced, and each traced segment also gets seven
 * values, taken by the workgroup's first thread: five timestamps of the
 * device's constant-rate real-time clock (skgemm_realtime_hz ticks per
 * second) {segment start, MAC loop done, partial stores and ready flags
 * done, fix-up waits done, segment done}, then the shader-clock counter at
 * the segment's start and at its end (so (v6 - v5) / (v4 - v0) times
 * skgemm_realtime_hz is the shader clock under the launch's own load).
 * times is device memory of 7 * trace_records uint64 values, laid out like
 * the records (record i's values at 7 * i).  The gap between the third and
 * fourth stamp is the time a workgroup spent waiting for its peers' partial
 * tiles (the Wait of the basic Stream-K algorithm); it is zero for segments
 * that wait for nobody. */
skgemm_status_t skgemm_run_timed(skgemm_plan_t plan,
                                 const void* A, int64_t lda, const void* B, int64_t ldb,
                                 void* C, int64_t ldc, float alpha, float beta,
                                 const float* scale_a, const float* scale_b,
                                 void* workspace, size_t ws_bytes,
                                 int32_t* trace, uint64_t* times, size_t trace_records, hipStream_t stream);

/* Ticks per second of the real-time clock skgemm_run_timed reads (current device). */
skgemm_status_t skgemm_realtime_hz(int64_t* hz);

/* Resolved plan, for logging and for comparing with an independent
 * enumerator of the schedule.  info[] receives, in order:
 *   0 M', 1 N', 2 K (problem as launched: M' = N and N' = M when C is
 *     column-major and the operands were swapped), 3 swapped (0/1),
 *   4 BM, 5 BN, 6 BK, 7 tiles_m, 8 tiles_n, 9 tiles, 10 iters_per_tile,
 *   11 policy (resolved skgemm_policy_t), 12 sk_tiles, 13 g_sk, 14 grid,
 *   15 sk_first (0/1), 16 p (co-resident workgroups), 17 hybrid_min_waves,
 *   18 A K-contiguous (0/1), 19 B K-contiguous (0/1), 20 G (problems of a
 *   grouped plan, 0 for one GEMM; fields 0-2, 7, 8 and 10 are 0 then and
 *   field 9 is the total tile count), 21 share (skgemm_share_t), 22 shares per
 * tile under the split fix-up (0 = owner fix-up), 23 workgroups per CU
 * (p = CUs * field 23), 24 wavefronts per workgroup, 25 batch (1 unless a
 * strided batched plan, whose fields 7 and 8 describe one problem and
 * field 9 counts the tiles of the whole batch), 26 / 27 the launched A / B is
 * copied to 128-byte aligned lines when passed misaligned (0/1), 28 bytes of
 * the fix-up part of the workspace, 29 LDS stages of the kernel's MAC-loop
 * pipeline (k-slabs in flight = stages - 1).
 * n is the capacity of info; up to 30 values are written. */
skgemm_status_t skgemm_plan_info(skgemm_plan_t plan, int64_t* info, int32_t n);

/* Analytical grid-size model constants (Analytical Modeling subsection)
 * used by the plan for its dtype and tile: time = a + b*[peers > 1] +
 * c*iters_per_cta + d*(peers - 1), microseconds.  e is the time of one
 * iteration on a CU that runs two workgroups: the automatic policy's split
 * choice uses e instead of c for grids larger than the CU count (p divided
 * by the occupancy, plan_info field 23).  Writes 5 doubles: a, b, c, d, e. */
skgemm_status_t skgemm_model_constants(skgemm_plan_t plan, double* abcde);

/* Host-side copy of the schedule the plan launches, in the same record
 * format as skgemm_run_traced (no device access). */
skgemm_status_t skgemm_schedule(skgemm_plan_t plan, int32_t* records, size_t cap, size_t* n);

/* ---------------------------------------------------------------- grouped GEMM
 * Several independent problems in ONE persistent launch: the problems' tiles
 * and MAC-loop iterations are concatenated (problem 0 first) into a single
 * iteration space, which the same policies split over the grid exactly as for
 * one GEMM (a Stream-K share may cross from one problem into the next).  All
 * problems share layouts and dtypes; each has its own M, N, K, pointers,
 * leading dimensions, alpha and beta.  K must be > 0 for every problem with
 * M, N > 0.  The run is a single kernel launch reading a device table, so it
 * can be captured in a HIP graph and replayed. */
typedef struct {
    const void* A;
    const void* B;
    void* C;
    int64_t lda, ldb, ldc;
    float alpha, beta;
} skgemm_group_args_t;

skgemm_status_t skgemm_grouped_plan(skgemm_plan_t* out, int32_t G, const int64_t* M, const int64_t* N,
                                    const int64_t* K, skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc,
                                    skgemm_dtype_t ta, skgemm_dtype_t tb, skgemm_dtype_t tc,
                                    const skgemm_options_t* opt);

/* Bytes of the per-problem table a grouped run reads (128 bytes per problem). */
skgemm_status_t skgemm_grouped_table_size(skgemm_plan_t plan, size_t* bytes);

/* Validates args[0..G) (host array, device pointers inside) and writes the
 * table into host memory `table` (at least skgemm_grouped_table_size bytes);
 * the caller copies it to device memory once and may reuse it for many runs
 * while the pointers stay valid. */
skgemm_status_t skgemm_grouped_table(skgemm_plan_t plan, const skgemm_group_args_t* args, void* table,
                                     size_t bytes);

/* One persistent launch over all problems; table_dev is the table in device
 * memory; workspace as for skgemm_run (skgemm_workspace_size of this plan). */
skgemm_status_t skgemm_grouped_run(skgemm_plan_t plan, const void* table_dev, void* workspace, size_t ws_bytes,
                                   hipStream_t stream);

/* Same, writing schedule records as skgemm_run_traced does (tile = global
 * tile index: problem i's tiles follow those of problems 0..i-1). */
skgemm_status_t skgemm_grouped_run_traced(skgemm_plan_t plan, const void* table_dev, void* workspace,
                                          size_t ws_bytes, int32_t* trace, size_t trace_records,
                                          hipStream_t stream);

/* ---------------------------------------------------------------- strided batched GEMM
 * batch equal problems C_i = alpha * s_A * s_B * A_i * B_i + beta * C_i,
 * i = 0 .. batch-1, whose operands lie at fixed element strides from the
 * first problem's (A_i = A + i * stride_a, and so on): one persistent launch
 * over the concatenated iteration space (problem 0's tiles first), split by
 * the same policies as one GEMM (the generalisation of Stream-K to other
 * GEMM-like problems the conclusion of the Stream-K chapter points to).  No
 * table: the kernel finds a tile's problem by one division.  Layouts, types,
 * options and workspace as for skgemm_plan / skgemm_run; plan_info field 25
 * is the batch.  Strides are non-negative element counts; stride_c must keep
 * consecutive C matrices apart (at least one C's extent) when batch > 1. */
skgemm_status_t skgemm_batched_plan(skgemm_plan_t* out, int64_t batch, int64_t M, int64_t N, int64_t K,
                                    skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc,
                                    skgemm_dtype_t ta, skgemm_dtype_t tb, skgemm_dtype_t tc,
                                    const skgemm_options_t* opt);
skgemm_status_t skgemm_batched_run(skgemm_plan_t plan,
                                   const void* A, int64_t lda, int64_t stride_a,
                                   const void* B, int64_t ldb, int64_t stride_b,
                                   void* C, int64_t ldc, int64_t stride_c, float alpha, float beta,
                                   const float* scale_a, const float* scale_b,
                                   void* workspace, size_t ws_bytes, hipStream_t stream);
/* Same, writing schedule records as skgemm_run_traced does (tile = global
 * tile index: problem i's tiles are i * tiles_per_problem onwards). */
skgemm_status_t skgemm_batched_run_traced(skgemm_plan_t plan,
                                          const void* A, int64_t lda, int64_t stride_a,
                                          const void* B, int64_t ldb, int64_t stride_b,
                                          void* C, int64_t ldc, int64_t stride_c, float alpha, float beta,
                                          const float* scale_a, const float* scale_b,
                                          void* workspace, size_t ws_bytes,
                                          int32_t* trace, size_t trace_records, hipStream_t stream);

/* ---------------------------------------------------------------- implicit-GEMM convolution
 * 2-D convolution (cross-correlation, as deep-learning frameworks define it)
 *   y[n,p,q,k] = alpha * sum_{r,s,c} x[n, p*stride_h + r*dil_h - pad_h, q*stride_w + s*dil_w - pad_w, c]
 *                        * w[k,r,s,c] + beta * y[n,p,q,k]
 * with x NHWC, w KRSC and y NPQK (channels innermost, dense), zero outside
 * the image, P = (h + 2 pad_h - dil_h (r - 1) - 1) / stride_h + 1 and Q
 * likewise: the GEMM with M = n P Q output pixels, N = k output channels and
 * K = r s c, whose A is gathered from x on the fly (implicit GEMM), split by
 * the same Stream-K schedules (the conclusion of the Stream-K chapter names
 * convolution among the GEMM-like problems the decomposition extends to).
 * 16-bit inputs, FP32 accumulation, output 16-bit (the input type) or FP32;
 * c must be a multiple of 64 and x at most 2^31 - 1 bytes
 * (SKGEMM_ERR_UNSUPPORTED otherwise).  plan_info describes the GEMM view;
 * workspace and options as for skgemm_plan / skgemm_run (the tile options
 * name 256x256x64, 128x128x64 or 256x64x64; the last is picked automatically
 * only for at most 64 output channels). */
typedef struct {
    int32_t n, h, w, c;                       /* input */
    int32_t k, r, s;                          /* filters: k output channels, r x s window */
    int32_t pad_h, pad_w, stride_h, stride_w, dil_h, dil_w;
} skgemm_conv_t;

skgemm_status_t skgemm_conv_plan(skgemm_plan_t* out, const skgemm_conv_t* conv, skgemm_dtype_t t_in,
                                 skgemm_dtype_t t_out, const skgemm_options_t* opt);
skgemm_status_t skgemm_conv_run(skgemm_plan_t plan, const void* x, const void* w, void* y, float alpha, float beta,
                                void* workspace, size_t ws_bytes, hipStream_t stream);
/* Same, writing schedule records as skgemm_run_traced does (tiles of the GEMM view). */
skgemm_status_t skgemm_conv_run_traced(skgemm_plan_t plan, const void* x, const void* w, void* y, float alpha,
                                       float beta, void* workspace, size_t ws_bytes, int32_t* trace,
                                       size_t trace_records, hipStream_t stream);

/* ---------------------------------------------------------------- FP8 front end
 * Per-tensor E4M3 quantisation of a rows x cols matrix X (FP32, BF16 or
 * FP16, layout lx, leading dimension ldx) into Q (E4M3FN bytes, layout lq,
 * leading dimension ldq; lq may differ from lx, e.g. to produce the
 * column-major B the FP8 GEMM needs):
 *   *scale = absmax(X) / 448 rounded to FP32, the maximum taken over the
 *            finite entries (1 if none of them is nonzero),
 *   Q = round-to-nearest-even E4M3 of clamp(X / scale, -448, 448), the
 *       quotient rounded to FP32; a NaN or infinite entry gives the NaN
 *       code 0x7f with the entry's sign (E4M3FN has no infinity), so it
 *       reaches the product as NaN.
 * scale is one FP32 on the device, to be passed as scale_a / scale_b of the
 * FP8 GEMM.  workspace: device scratch of skgemm_quantize_workspace_size
 * bytes, 4-byte aligned, no initialisation needed.  Asynchronous on stream:
 * two kernel launches (an absmax pass, then a quantising pass that reduces
 * the maxima itself), or three when the quantising grid exceeds 4096
 * workgroups (a one-workgroup reduction between them); an empty X gives
 * scale = 1 (two launches). */
skgemm_status_t skgemm_quantize_workspace_size(size_t* bytes);
skgemm_status_t skgemm_quantize_e4m3(const void* X, skgemm_dtype_t tx, int64_t rows, int64_t cols,
                                     skgemm_layout_t lx, int64_t ldx, void* Q, skgemm_layout_t lq, int64_t ldq,
                                     float* scale, void* workspace, size_t ws_bytes, hipStream_t stream);

/* Reads the workspace's error word (synchronises the stream).  Returns
 * SKGEMM_ERR_TIMEOUT if a fix-up wait expired in an earlier run. */
skgemm_status_t skgemm_check_device_error(const void* workspace, hipStream_t stream);

skgemm_status_t skgemm_plan_destroy(skgemm_plan_t plan);

const char* skgemm_status_string(skgemm_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* SKGEMM_H */
