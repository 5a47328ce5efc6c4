// Host side of skgemm: argument checks, the planner (iteration space, policy,
// grid size, workspace) and the C ABI declared in include/skgemm.h.
//
// Planning follows the Kernel Configuration and Data-parallel Hybridization
// subsections: one tile configuration per input type, the grid of persistent
// workgroups sized to the co-resident capacity p = CUs x occupancy, and the
// policy resolved from the number of full data-parallel waves w = t / p and
// the remainder r = t mod p.  With fewer tiles than workgroups the grid size g
// is chosen by the analytical model of the Analytical Modeling subsection.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "skgemm.h"
#include "skgemm_internal.h"

using namespace skg;

struct skgemm_plan_s {
    // problem as given
    int64_t M, N, K;
    skgemm_layout_t la, lb, lc;
    skgemm_dtype_t ta, tc;
    // problem as launched (C column-major runs C^T = B^T A^T)
    bool swapped;
    int32_t Ml, Nl, Kl;
    bool akc, bkc;   // K-contiguity of the launched A and B
    int dtype, out;
    int variant;     // tile variant (0 default, 1 small 16-bit tile)
    // tiling and schedule
    int BM, BN, BK;
    int tm, tn, t, ipt;
    int policy;
    int sk_tiles, g_sk, grid;
    bool sk_first;
    int p, occ, hybrid_min_waves;   // p = CUs * occ co-resident workgroups
    int raster, xcds;  // tile raster group rows; XCD count for the workgroup permutation
    int spin_limit;    // polls before a fix-up wait gives up
    bool share_prop;   // proportional (else leading) even share
    bool fixup_owner;  // the owner alone reduces every split tile
    int coop_s;        // >= 2: split fix-up over tiles cut into coop_s one-segment shares
    int sk_q, sk_r;
    double model[5];   // a, b, c, d of the grid-size model; e: c with every workgroup slot busy
    // workspace layout
    size_t ws_bytes, flags_off, partials_off;
    // re-layout of the launched A (0) and B (1) into the workspace when their
    // lines are not 128-byte aligned (decided per call from the leading
    // dimension; planned only where the model says it pays)
    bool pack[2];
    int64_t pack_lines[2], pack_cols[2], pack_ld[2];
    size_t pack_off[2];
    size_t ws_total;                         // ws_bytes plus the re-layout regions
    int max_segs;
    // iteration space as problems (a single GEMM is one problem)
    int G;                                  // 0 for a single-GEMM plan
    std::vector<int32_t> pM, pN, pK, ptm, ptn, pipt;   // launched shapes
    std::vector<int32_t> tile_base;         // G + 1 prefix of tiles
    std::vector<int64_t> iter_base;         // G + 1 prefix of MAC-loop iterations
    std::vector<int64_t> gM, gN, gK;        // shapes as given, in iteration-space order
    std::vector<int32_t> order;             // caller's index of each problem in iteration-space order
    int t_work;                             // tiles with MAC-loop iterations (they come first)
    int64_t batch;                          // strided batch of equal problems (1 = one GEMM)
    bool conv;                              // implicit-GEMM convolution (tile variants 3, 4 and 7)
    ConvArgs cv;
    int64_t sk_iters;
};

namespace {

int elem_bytes(skgemm_dtype_t t) {
    switch (t) {
        case SKGEMM_F32: return 4;
        case SKGEMM_F16:
        case SKGEMM_BF16: return 2;
        case SKGEMM_F8E4M3: return 1;
        case SKGEMM_F64: return 8;
    }
    return 0;
}

int to_dt(skgemm_dtype_t t) {
    switch (t) {
        case SKGEMM_F32: return DT_F32;
        case SKGEMM_F16: return DT_F16;
        case SKGEMM_BF16: return DT_BF16;
        case SKGEMM_F8E4M3: return DT_F8;
        case SKGEMM_F64: return DT_F64;
    }
    return -1;
}

// Tile of each (input type, variant); {0, 0, 0} where the variant does not exist.
TileCfg tile_for(int dt, int v) {
    if (v == 0) {
        switch (dt) {
            case DT_F32: return kTileF32;
            case DT_F8: return kTileF8;
            case DT_F64: return kTileF64;
            default: return kTile16;
        }
    }
    if ((v == 1 || v == 2) && (dt == DT_BF16 || dt == DT_F16)) return kTile16S;
    if (v == 3 && (dt == DT_BF16 || dt == DT_F16)) return kTile16;     // convolution
    if (v == 4 && (dt == DT_BF16 || dt == DT_F16)) return kTile16S;
    if (v == 5 && (dt == DT_BF16 || dt == DT_F16)) return kTile16K;     // skinny
    if ((v == 6 || v == 7) && (dt == DT_BF16 || dt == DT_F16)) return kTile16T;     // tall
    if ((v == kVariantDeep || v == kVariantDeepConv) && (dt == DT_BF16 || dt == DT_F16)) return kTile16D;   // three stages
    if (v == 1 && dt == DT_F8) return kTileF8S;
    if (v == 1 && dt == DT_F64) return kTileF64L;
    return TileCfg{0, 0, 0};
}

// Grid-size model constants (a, b, c, d) per input type and tile variant, in
// microseconds measured on MI355X (paper_2212_08964_amd/calibrate.py): a the
// fixed cost of a workgroup's tile, b the cost of publishing a partial tile,
// c the cost of one MAC-loop iteration, d the cost of adding one peer's
// partial.  The grid-size argmin only depends on their ratios; the absolute
// values let the planner compare tile variants.
void model_for(int dt, int v, double* m) {
    // a-d: least-squares fits over tile-aligned grids of at most one
    // workgroup per CU (calibrate.py); e: the per-iteration time of one
    // workgroup when all p co-resident workgroups run (a data-parallel problem
    // of several full waves), used for grids larger than the CU count and in
    // the comparison of tile variants.  FP8 shares the 16-bit constants of
    // the same tile size: same wave layout, twice the k per iteration at
    // twice the MFMA rate.
    if (dt == DT_F64 && v == 1) { m[0] = 7.98; m[1] = 1.22; m[2] = 2.04; m[3] = 1.13; m[4] = 3.84; return; }
    if (dt == DT_F64) { m[0] = 5.00; m[1] = 1.23; m[2] = 0.713; m[3] = 1.13; m[4] = 2.09; return; }
    if (dt == DT_F32) { m[0] = 6.20; m[1] = 1.25; m[2] = 2.07; m[3] = 0.569; m[4] = 3.99; return; }
    // the convolution variants take the constants of the GEMM tile of their shape
    // the three-stage small tile: calibrate.py's grid mode with e from one
    // full wave of it (one workgroup per CU)
    if (v == kVariantDeep || v == kVariantDeepConv) { m[0] = 5.98; m[1] = 1.21; m[2] = 0.581; m[3] = 0.658; m[4] = 0.608; return; }
    if (v == 2) { m[0] = 5.38; m[1] = 1.51; m[2] = 0.583; m[3] = 0.648; m[4] = 0.981; return; }
    if (v == 1 || v == 4) { m[0] = 5.60; m[1] = 1.38; m[2] = 0.603; m[3] = 0.577; m[4] = 0.899; return; }
    if (v == 5) { m[0] = 5.99; m[1] = 1.49; m[2] = 0.703; m[3] = 0.570; m[4] = 1.009; return; }
    if (v == 6 || v == 7) { m[0] = 5.28; m[1] = 1.87; m[2] = 0.716; m[3] = 0.551; m[4] = 1.009; return; }
    m[0] = 9.88; m[1] = 2.78; m[2] = 1.351; m[3] = 0.941; m[4] = 1.693;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// HBM bytes per microsecond a kernel of this library can stream: 6 TB/s, 75 %
// of MI355X's 8 TB/s, the rate its HBM-bound FP8 quantising passes reach.
constexpr double kHbmBytesPerUs = 6.0e6;

double model_time(int64_t g, int64_t t, int64_t ipt, const double* m) {
    const int64_t ipc = cdiv(t * ipt, g);
    const int64_t peers = cdiv(ipt, ipc);
    return m[0] + m[1] * (peers > 1 ? 1.0 : 0.0) + m[2] * double(ipc) + m[3] * double(peers - 1);
}

int model_best_g(int64_t t, int64_t ipt, int64_t p, const double* m) {
    int64_t best_g = t;
    double best = 0.0;
    for (int64_t g = t; g <= std::max(t, p); ++g) {
        const double v = model_time(g, t, ipt, m);
        if (g == t || v < best) {
            best = v;
            best_g = g;
        }
    }
    return int(best_g);
}

// Split factor s in [1, min(p / t, ipt)] that minimises the modelled time of
// basic Stream-K over t tiles with g = s * t (the smallest s on ties).  A grid
// larger than the CU count puts n = ceil(g / cus) workgroups on some CUs, and
// those run an iteration in c + (e - c)(n - 1)/(occ - 1) rather than c (e,
// m[4], with all occ = p / cus slots of a CU busy): the slowest workgroup
// sets the time.  On problems without ragged edges (M, N, K multiples of 64)
// a grid above the CU count with three or more shares per tile needs at
// least 8 iterations per share: there the data-parallel tiles run at their
// calibrated speed, and short shares on CUs holding two workgroups lost to
// data-parallel in every measured case (BF16 sweep: 0.81-0.97x at 100-165
// tiles of 128x128 with 4-6 iterations per share), a cost of the fix-up
// traffic and co-residency the per-workgroup model does not see.
//
// Memory-bound regime: no split can run faster than its HBM traffic allows,
// the operands' bytes plus the partial tiles the split writes and reads back
// (2 (s - 1) t tile_bytes), at kHbmBytesPerUs; the modelled time of a split is
// the larger of the two (ties still go to the smallest s).
int model_best_split(int64_t t, int64_t ipt, int64_t p, int64_t cus, const double* m, bool aligned,
                     double op_bytes, double tile_bytes) {
    const int64_t smax = std::max<int64_t>(1, std::min(p / std::max<int64_t>(t, 1), ipt));
    const int64_t occ = std::max<int64_t>(1, p / std::max<int64_t>(cus, 1));
    auto time_at = [&](int64_t g) {
        const int64_t n = cdiv(g, cus);
        const double c = n <= 1 || occ <= 1 ? m[2] : m[2] + (m[4] - m[2]) * double(n - 1) / double(occ - 1);
        const double mg[4] = {m[0], m[1], c, m[3]};
        const double partials = 2.0 * double(g - t) * tile_bytes;
        return std::max(model_time(g, t, ipt, mg), (op_bytes + partials) / kHbmBytesPerUs);
    };
    int best_s = 1;
    double best = time_at(t);
    for (int64_t sp = 2; sp <= smax; ++sp) {
        if (aligned && sp > 2 && t * sp > cus && cdiv(ipt, sp) < 8) break;
        const double v = time_at(t * sp);
        if (v < best) {
            best = v;
            best_s = int(sp);
        }
    }
    return best_s;
}

// First iteration of workgroup x's even share of `total` iterations over g
// workgroups: proportional (floor(x * total / g)) or leading (the first
// total mod g workgroups get one iteration more).
int share_start(int x, int64_t total, int g, bool prop) {
    if (prop) return int(int64_t(x) * total / g);
    const int64_t q = total / g, r = total % g;
    return int(x * q + std::min<int64_t>(x, r));
}

// Workgroup whose share holds iteration i.
int owner_of(int i, int64_t total, int g, bool prop) {
    if (prop) return int((int64_t(i + 1) * g - 1) / total);
    const int64_t q = total / g, r = total % g;
    return int((i < r * (q + 1)) ? i / (q + 1) : r + (i - r * (q + 1)) / q);
}

int find_last_le(const std::vector<int64_t>& base, int G, int64_t x) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int find_last_le32(const std::vector<int32_t>& base, int G, int x) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Walks the schedule of workgroup x exactly as the kernel does; calls
// emit(seq, global_tile, lo, hi, role, first_peer, last_peer) per segment.
template <class F>
int walk(const skgemm_plan_s& pl, int x, F&& emit) {
    const int np = int(pl.pipt.size());
    int sk_it = 0, sk_end = 0;
    if (x < pl.g_sk) {
        sk_it = share_start(x, pl.sk_iters, pl.g_sk, pl.share_prop);
        sk_end = share_start(x + 1, pl.sk_iters, pl.g_sk, pl.share_prop);
    }
    int dp_tile = pl.sk_tiles + x;
    int seq = 0;
    for (;;) {
        const bool sk_left = sk_it < sk_end, dp_left = dp_tile < pl.t;
        if (!sk_left && !dp_left) break;
        const bool take_sk = pl.sk_first ? sk_left : !dp_left;
        int gtile, lo, hi, role, p0 = -1, p1 = -1;
        if (take_sk) {
            const int pi = find_last_le(pl.iter_base, np, sk_it);
            const int ipt = pl.pipt[pi];
            const int tile = int((sk_it - pl.iter_base[pi]) / ipt);
            const int first = int(pl.iter_base[pi]) + tile * ipt, last = first + ipt;
            gtile = pl.tile_base[pi] + tile;
            lo = sk_it - first;
            hi = std::min(sk_end, last) - first;
            if (sk_it != first) {
                role = ROLE_PARTIAL;
            } else if (sk_end < last) {
                role = ROLE_OWNER;
                p0 = x + 1;
                p1 = owner_of(last - 1, pl.sk_iters, pl.g_sk, pl.share_prop);
            } else {
                role = ROLE_FULL;
            }
            sk_it = last;
        } else {
            gtile = dp_tile;
            lo = 0;
            hi = pl.pipt[find_last_le32(pl.tile_base, np, dp_tile)];
            role = ROLE_FULL;
            dp_tile += pl.grid;
        }
        emit(seq, gtile, lo, hi, role, p0, p1);
        ++seq;
    }
    return seq;
}

struct DevInfo {
    int cus = 0;
    int occ[kDTypes][2][2][kVariants] = {};
    bool have_occ[kDTypes][2][2][kVariants] = {};
};
std::mutex g_dev_mu;
DevInfo g_dev[64];

skgemm_status_t device_capacity(int dt, bool akc, bool bkc, int v, int* cus, int* occ) {
    if (dt < 0 || dt >= kDTypes || v < 0 || v >= kVariants) return SKGEMM_ERR_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SKGEMM_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DevInfo& d = g_dev[dev];
    if (d.cus == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            return SKGEMM_ERR_HIP;
        d.cus = n;
    }
    if (!d.have_occ[dt][akc][bkc][v]) {
        const int o = kernel_occupancy(dt, akc, bkc, v);
        if (o <= 0) return SKGEMM_ERR_HIP;
        d.occ[dt][akc][bkc][v] = o;
        d.have_occ[dt][akc][bkc][v] = true;
    }
    *cus = d.cus;
    *occ = d.occ[dt][akc][bkc][v];
    return SKGEMM_OK;
}

constexpr int64_t kMaxDim = (int64_t(1) << 31) - 1;
// Tile raster groups of 8 tile rows: 8 x 4 (256-wide tiles, one workgroup per
// CU) or 8 x 8 (128-wide, two per CU) neighbouring tiles per XCD at a time.
constexpr int kDefaultRaster = 8, kMaxRaster = 1 << 16;
// MI355X hands workgroups round-robin to its 8 XCDs.
constexpr int kDefaultXcds = 8, kMaxXcds = 64;
// Polls of a ready flag before a fix-up wait gives up (each poll sleeps about
// 128 clocks: well over a second in all, against microseconds for a hand-off).
constexpr int kDefaultSpinLimit = 1 << 22;

}  // namespace

extern "C" {

void skgemm_default_options(skgemm_options_t* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->policy = SKGEMM_POLICY_AUTO;
    opt->hybrid_min_waves = 2;
}

// Common part of single and grouped planning: validate the options, resolve
// the co-resident capacity, then the policy, Stream-K region, grid and
// workspace for the iteration space in pl->{pipt, tile_base, iter_base}.
// Every problem with tiles has the same iterations per tile (a single GEMM
// always does), so shares can line up with tile seams.
static bool uniform_ipt(const skgemm_plan_s& pl) {
    int ipt = -1;
    for (size_t i = 0; i < pl.pipt.size(); ++i) {
        if (pl.tile_base[i + 1] == pl.tile_base[i] || pl.pipt[i] == 0) continue;
        if (ipt < 0) ipt = pl.pipt[i];
        else if (pl.pipt[i] != ipt) return false;
    }
    return true;
}

// Algorithmic HBM bytes of a plan's problems: A and B read once, C written
// once (a strided batch counts every problem).
static double operand_bytes(const skgemm_plan_s& pl) {
    const double eb = elem_bytes(pl.ta), ec = elem_bytes(pl.tc);
    double sum = 0.0;
    for (size_t i = 0; i < pl.pM.size(); ++i)
        sum += (double(pl.pM[i]) * pl.pK[i] + double(pl.pK[i]) * pl.pN[i]) * eb + double(pl.pM[i]) * pl.pN[i] * ec;
    return sum * double(pl.batch > 0 ? pl.batch : 1);
}

static skgemm_status_t finish_plan(skgemm_plan_s* pl, const skgemm_options_t& o) {
    int cus = o.num_cus, occ = o.occupancy;
    if (cus == 0 || occ == 0) {
        int qc = 0, qo = 0;
        const skgemm_status_t st = device_capacity(pl->dtype, pl->akc, pl->bkc, pl->variant, &qc, &qo);
        if (st != SKGEMM_OK) return st;
        if (cus == 0) cus = qc;
        if (occ == 0) occ = qo;
    }
    const int64_t p = int64_t(cus) * occ;
    if (p <= 0 || p > kMaxDim) return SKGEMM_ERR_INVALID_ARG;
    pl->p = int(p);
    pl->occ = occ;
    const int np = int(pl->pipt.size());
    const int64_t t = pl->tile_base[np];
    const int64_t total = pl->iter_base[np];
    if (t > kMaxDim || total > kMaxDim) return SKGEMM_ERR_UNSUPPORTED;
    pl->t = int(t);
    // Tiles of K = 0 problems (epilogue only, C = beta * C) come after every
    // tile with iterations and are never part of the Stream-K region: the
    // policies split the first t_work tiles, and the rest run as
    // data-parallel tiles.
    int64_t t_work = t;
    for (int i = 0; i < np; ++i)
        if (pl->pipt[i] == 0 && pl->tile_base[i + 1] > pl->tile_base[i]) {
            t_work = pl->tile_base[i];
            break;
        }
    pl->t_work = int(t_work);
    // iterations per tile for the model (their mean over a grouped launch)
    const int64_t ipt = t_work ? (total + t_work - 1) / t_work : 0;
    int policy = o.policy;
    int auto_g = 0;
    pl->sk_tiles = 0; pl->g_sk = 0; pl->grid = 0; pl->sk_first = true;
    if (t > 0) {
        if (total == 0) policy = SKGEMM_POLICY_DP;    // K == 0: epilogue-only tiles
        const int64_t w = t_work / p, r = t_work % p;
        if (policy == SKGEMM_POLICY_AUTO && !uniform_ipt(*pl)) policy = SKGEMM_POLICY_PAPER;
        if (policy == SKGEMM_POLICY_PAPER) {
            // the paper's selection from the full waves w and the remainder r
            if (r == 0) policy = SKGEMM_POLICY_DP;
            else if (w == 0) policy = SKGEMM_POLICY_SK;
            else if (w >= pl->hybrid_min_waves) policy = SKGEMM_POLICY_2TILE_SK_DP;
            else policy = SKGEMM_POLICY_DP_1TILE_SK;
        } else if (policy == SKGEMM_POLICY_AUTO) {
            if (r == 0) {
                policy = SKGEMM_POLICY_DP;
            } else if (w >= kAutoMaxWaves) {
                // enough whole waves that the remainder is a small part of the
                // time: persistent workgroups with a fixed share of
                // data-parallel tiles lose more to their uneven progress than
                // a split remainder gains (FP64 8192^3: -5 %)
                policy = SKGEMM_POLICY_DP;
            } else {
                // Tile-aligned split of the remainder: with g = s * (its tile
                // count) and proportional shares, every tile is cut into s
                // parts at the same k-offsets, so the workgroups of an XCD
                // stream the same k-slabs at the same time and share them in
                // L2.  Unaligned shares start each workgroup at its own
                // k-offset, which on MI355X's per-XCD L2 costs up to 2x.
                const int64_t sk_t = w == 0 ? t_work : r;
                bool aligned = true;
                for (size_t i = 0; i < pl->pM.size(); ++i)
                    aligned = aligned && pl->pM[i] % 64 == 0 && pl->pN[i] % 64 == 0 && pl->pK[i] % 64 == 0;
                // the HBM bound of the split region: its tiles' share of the
                // operand bytes (the data-parallel waves before it stream theirs)
                const double op_sk = operand_bytes(*pl) * double(sk_t) / double(t_work);
                const int s_best = model_best_split(sk_t, ipt, p, cus, pl->model, aligned, op_sk,
                                                    double(pl->BM) * pl->BN * (pl->dtype == DT_F64 ? 8 : 4));
                if (s_best == 1) policy = SKGEMM_POLICY_DP;
                else {
                    policy = w == 0 ? SKGEMM_POLICY_SK : SKGEMM_POLICY_DP_1TILE_SK;
                    auto_g = int(sk_t * s_best);
                }
            }
        }
        if (policy == SKGEMM_POLICY_DP) {
            pl->grid = int(t);
        } else {
            if (policy == SKGEMM_POLICY_SK) {
                pl->sk_tiles = int(t_work);
            } else if (policy == SKGEMM_POLICY_DP_1TILE_SK) {
                pl->sk_tiles = int(r);
                pl->sk_first = false;
            } else {
                pl->sk_tiles = int(w == 0 ? t_work : r + p);
            }
            // iterations of the Stream-K region [0, sk_tiles)
            const int pi = find_last_le32(pl->tile_base, np, pl->sk_tiles);
            pl->sk_iters = pl->sk_tiles >= t ? total
                                             : pl->iter_base[pi] + int64_t(pl->sk_tiles - pl->tile_base[pi]) * pl->pipt[pi];
            if (policy == SKGEMM_POLICY_SK) {
                if (o.force_g) pl->g_sk = o.force_g;
                else if (auto_g) pl->g_sk = auto_g;
                else if (t_work >= p) pl->g_sk = int(p);
                else pl->g_sk = model_best_g(t_work, ipt, p, pl->model);
                pl->grid = pl->g_sk;
            } else {
                if (pl->sk_tiles)
                    pl->g_sk = o.force_g ? o.force_g : auto_g ? auto_g : int(std::min<int64_t>(p, pl->sk_iters));
                pl->grid = (t - pl->sk_tiles > 0) ? int(p) : pl->g_sk;
                pl->grid = std::max(pl->grid, pl->g_sk);
            }
        }
    }
    pl->policy = policy;
    // A forced grid beyond the Stream-K iterations would leave workgroups
    // with empty shares (between peers, under the proportional share): use
    // one workgroup per iteration at most.
    if (pl->g_sk > pl->sk_iters) pl->g_sk = int(pl->sk_iters);
    if (pl->policy == SKGEMM_POLICY_SK) pl->grid = pl->g_sk;
    else if (pl->g_sk) pl->grid = std::max(pl->grid, pl->g_sk);
    // Owners wait on workgroups with higher indices, so every Stream-K
    // workgroup must be resident at once.
    if (pl->g_sk > pl->p || pl->g_sk > kMaxFlagLines) return SKGEMM_ERR_CAPACITY;
    if (pl->g_sk) {
        pl->sk_q = int(pl->sk_iters / pl->g_sk);
        pl->sk_r = int(pl->sk_iters % pl->g_sk);
    }
    // Split fix-up: a single GEMM whose Stream-K tiles are each cut into s
    // shares that start and end on the tile, so each Stream-K workgroup
    // performs exactly one segment: g = s * tiles and, with the proportional
    // share (workgroup x starts at floor(x * ipt / s) within tile x / s), any
    // s <= ipt; with the leading share s must divide ipt.
    pl->coop_s = 0;
    if (!pl->fixup_owner && pl->pM.size() == 1 && pl->g_sk && pl->sk_tiles && pl->g_sk % pl->sk_tiles == 0) {
        const int s = pl->g_sk / pl->sk_tiles, ipt = pl->pipt[0];
        if (s >= 2 && s <= ipt && (pl->share_prop || ipt % s == 0)) pl->coop_s = s;
    }
    pl->flags_off = kWsHeaderBytes;
    pl->partials_off = (kWsHeaderBytes + size_t(kMaxFlagLines) * kFlagStrideInts * 4 + 255) & ~size_t(255);
    // partial tiles accumulate in FP32, or FP64 for FP64 inputs
    const size_t acc_bytes = pl->dtype == DT_F64 ? 8 : 4;
    pl->ws_bytes = pl->g_sk ? pl->partials_off + size_t(pl->g_sk) * pl->BM * pl->BN * acc_bytes : 0;
    pl->pack[0] = pl->pack[1] = false;
    pl->ws_total = pl->ws_bytes;
    int mx = 0;
    for (int x = 0; x < pl->grid; ++x) mx = std::max(mx, walk(*pl, x, [](int, int, int, int, int, int, int) {}));
    pl->max_segs = mx;
    return SKGEMM_OK;
}

// Checks shared by single and grouped plans; fills dtype, layout and tile
// fields of pl.
static skgemm_status_t init_common(skgemm_plan_s* pl, skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc,
                                   skgemm_dtype_t ta, skgemm_dtype_t tb, skgemm_dtype_t tc,
                                   const skgemm_options_t& o) {
    if ((la != SKGEMM_ROW_MAJOR && la != SKGEMM_COL_MAJOR) || (lb != SKGEMM_ROW_MAJOR && lb != SKGEMM_COL_MAJOR) ||
        (lc != SKGEMM_ROW_MAJOR && lc != SKGEMM_COL_MAJOR))
        return SKGEMM_ERR_INVALID_ARG;
    if (to_dt(ta) < 0 || to_dt(tb) < 0 || to_dt(tc) < 0) return SKGEMM_ERR_INVALID_ARG;
    if (ta != tb) return SKGEMM_ERR_UNSUPPORTED;
    if (tc == SKGEMM_F8E4M3) return SKGEMM_ERR_UNSUPPORTED;
    if (ta != SKGEMM_F8E4M3 && ta != SKGEMM_F32 && tc != ta && tc != SKGEMM_F32) return SKGEMM_ERR_UNSUPPORTED;
    if (ta == SKGEMM_F32 && tc != SKGEMM_F32) return SKGEMM_ERR_UNSUPPORTED;
    if ((ta == SKGEMM_F64) != (tc == SKGEMM_F64)) return SKGEMM_ERR_UNSUPPORTED;
    if (o.force_g < 0 || o.num_cus < 0 || o.occupancy < 0 || o.tile_waves < 0 || o.spin_limit < 0)
        return SKGEMM_ERR_INVALID_ARG;
    if (o.raster_rows < 0 || o.raster_rows > kMaxRaster || o.xcds < 0 || o.xcds > kMaxXcds)
        return SKGEMM_ERR_INVALID_ARG;
    if (o.policy < SKGEMM_POLICY_AUTO || o.policy > SKGEMM_POLICY_PAPER) return SKGEMM_ERR_INVALID_ARG;
    pl->la = la; pl->lb = lb; pl->lc = lc;
    pl->ta = ta; pl->tc = tc;
    pl->dtype = to_dt(ta);
    pl->out = to_dt(tc);
    pl->swapped = (lc == SKGEMM_COL_MAJOR);
    const bool a_kc = (la == SKGEMM_ROW_MAJOR), b_kc = (lb == SKGEMM_COL_MAJOR);
    pl->akc = pl->swapped ? b_kc : a_kc;
    pl->bkc = pl->swapped ? a_kc : b_kc;
    if (!kernel_exists(pl->dtype, pl->akc, pl->bkc, 0)) return SKGEMM_ERR_UNSUPPORTED;
    pl->hybrid_min_waves = o.hybrid_min_waves;
    if (o.share != SKGEMM_SHARE_PROPORTIONAL && o.share != SKGEMM_SHARE_LEADING) return SKGEMM_ERR_INVALID_ARG;
    if (o.fixup != SKGEMM_FIXUP_AUTO && o.fixup != SKGEMM_FIXUP_OWNER) return SKGEMM_ERR_INVALID_ARG;
    if (o.relayout < -1 || o.relayout > 3) return SKGEMM_ERR_INVALID_ARG;
    pl->fixup_owner = o.fixup == SKGEMM_FIXUP_OWNER;
    pl->share_prop = o.share == SKGEMM_SHARE_PROPORTIONAL;
    pl->raster = o.raster_rows ? o.raster_rows : kDefaultRaster;
    pl->xcds = o.xcds ? o.xcds : kDefaultXcds;
    pl->spin_limit = o.spin_limit ? o.spin_limit : kDefaultSpinLimit;
    return SKGEMM_OK;
}

static void add_problem(skgemm_plan_s* pl, int64_t M, int64_t N, int64_t K);

// Modelled runtime (microseconds) of a resolved plan, by the analytical model
// of the Analytical Modeling subsection extended to the hybrids: a
// workgroup's Stream-K share plus its data-parallel tiles, each tile paying
// the fixed cost a; pure data-parallel plans run in ceil(t / p) waves.
static double plan_estimate_compute(const skgemm_plan_s* pl);

// The larger of the compute model's time and the plan's HBM time (operand
// bytes plus partial tiles written and read back).
static double plan_estimate(const skgemm_plan_s* pl, double* compute) {
    const double tc = plan_estimate_compute(pl);
    if (compute) *compute = tc;
    if (pl->t == 0) return 0.0;
    const double partials = 2.0 * double(pl->g_sk > pl->sk_tiles ? pl->g_sk - pl->sk_tiles : 0) * pl->BM * pl->BN *
                            (pl->dtype == DT_F64 ? 8.0 : 4.0);
    return std::max(tc, (operand_bytes(*pl) + partials) / kHbmBytesPerUs);
}

static double plan_estimate_compute(const skgemm_plan_s* pl) {
    if (pl->t == 0) return 0.0;
    const int np = int(pl->pipt.size());
    const double ipt = double(pl->iter_base[np]) / pl->t;
    const double* m = pl->model;
    const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4];
    // per-iteration time with `active` of the p workgroup slots busy
    auto c_at = [&](int64_t active) { return c + (e - c) * std::min(1.0, double(active) / pl->p); };
    if (pl->g_sk == 0) {
        const int64_t full = pl->t / pl->p, rem = pl->t % pl->p;
        return double(full) * (a + e * ipt) + (rem ? a + c_at(rem) * ipt : 0.0);
    }
    const int64_t ipc = cdiv(pl->sk_iters, pl->g_sk);
    const int64_t peers = std::max<int64_t>(1, cdiv(int64_t(ipt + 0.5), ipc));
    const int64_t dp_per_wg = cdiv(pl->t - pl->sk_tiles, pl->grid);
    return a + double(dp_per_wg) * (a + e * ipt) + b * (peers > 1 ? 1.0 : 0.0) + c_at(pl->g_sk) * double(ipc) +
           d * double(peers - 1);
}

// Plan of tile variant v for the problems of base under options o; nullptr
// with *st set when the variant cannot run them (SKGEMM_ERR_HIP: out of
// host memory).  The three-stage small tile holds one workgroup per CU, so a
// co-residency given in the options counts as 1 for it.
static skgemm_plan_s* build_variant(const skgemm_plan_s* base, int v, const skgemm_options_t& o, int G,
                                    const int64_t* M, const int64_t* N, const int64_t* K, skgemm_status_t* st) {
    skgemm_options_t ov = o;
    if ((v == kVariantDeep || v == kVariantDeepConv) && ov.occupancy) ov.occupancy = 1;
    const TileCfg tc_ = tile_for(base->dtype, v);
    skgemm_plan_s* pl = new (std::nothrow) skgemm_plan_s(*base);
    if (!pl) {
        *st = SKGEMM_ERR_HIP;
        return nullptr;
    }
    pl->variant = v;
    pl->BM = tc_.bm; pl->BN = tc_.bn; pl->BK = tc_.bk;
    model_for(pl->dtype, v, pl->model);
    for (int j = 0; j < G; ++j) {
        const int i = pl->order[j];
        add_problem(pl, M[i], N[i], K[i]);
    }
    *st = SKGEMM_OK;
    if (!pl->G) {
        pl->Ml = pl->pM[0]; pl->Nl = pl->pN[0]; pl->Kl = int32_t(pl->K);
        pl->tm = pl->ptm[0]; pl->tn = pl->ptn[0]; pl->ipt = pl->pipt[0];
        const int64_t tiles = int64_t(pl->tm) * pl->tn * pl->batch;
        if (tiles > kMaxDim || tiles * pl->ipt > kMaxDim) {
            *st = SKGEMM_ERR_UNSUPPORTED;
        } else if (pl->batch > 1) {
            // a strided batch is one iteration space of batch * t1 tiles
            // (problem after problem), each with the same iterations
            pl->tile_base[1] = int32_t(tiles);
            pl->iter_base[1] = tiles * pl->ipt;
        }
    }
    if (*st == SKGEMM_OK) *st = finish_plan(pl, ov);
    if (*st != SKGEMM_OK) {
        delete pl;
        return nullptr;
    }
    return pl;
}

// Builds the plan for every admissible tile variant (the one the options
// name, else all that exist) and keeps the one with the smallest modelled
// runtime (the default tile on ties); the small 16-bit tile competes on its
// eight-wave layout (the four-wave one only where the options ask for it).
static skgemm_status_t plan_variants(skgemm_plan_s* base, const skgemm_options_t& o, int G, const int64_t* M,
                                     const int64_t* N, const int64_t* K, skgemm_plan_s** out) {
    const bool named = o.tile_m || o.tile_n || o.tile_k;
    skgemm_plan_s* cand[kVariants] = {};
    skgemm_status_t last = SKGEMM_ERR_UNSUPPORTED;
    for (int v = 0; v < kVariants; ++v) {
        if (v == kVariantDeep || v == kVariantDeepConv) continue;   // substituted below, not candidates
        if (is_conv_variant(v) != base->conv) continue;     // the convolution kernels are variants 3, 4 and 7
        // the skinny tile only where every launched problem has at most its
        // 64 rows (unless the options name it)
        if (v == 5 && !named) {
            int64_t rows = 0;
            for (int j = 0; j < G; ++j) rows = std::max<int64_t>(rows, base->swapped ? N[j] : M[j]);
            if (rows > kTile16K.bm) continue;
        }
        // the tall tile likewise where every launched problem has at most its
        // 64 columns
        if ((v == 6 || v == 7) && !named) {
            int64_t cols = 0;
            for (int j = 0; j < G; ++j) cols = std::max<int64_t>(cols, base->swapped ? M[j] : N[j]);
            if (cols > kTile16T.bn) continue;
        }
        const TileCfg tc_ = tile_for(base->dtype, v);
        if (!tc_.bm || !kernel_exists(base->dtype, base->akc, base->bkc, v)) continue;
        if (named && ((o.tile_m && o.tile_m != tc_.bm) || (o.tile_n && o.tile_n != tc_.bn) ||
                      (o.tile_k && o.tile_k != tc_.bk)))
            continue;
        if (o.tile_waves && kernel_threads(base->dtype, v) != 64 * o.tile_waves) continue;
        skgemm_status_t st = SKGEMM_OK;
        skgemm_plan_s* pl = build_variant(base, v, o, G, M, N, K, &st);
        if (!pl) {
            if (st == SKGEMM_ERR_HIP) {
                for (skgemm_plan_s* c : cand) delete c;
                return st;
            }
            last = st;
            continue;
        }
        cand[v] = pl;
    }
    // The small 16-bit tile on eight waves runs data-parallel tiles 8 % and
    // split ones 3 % faster than on four (BF16 sweep), so it replaces the
    // four-wave tile.  Keeping the four-wave tile for split plans, whose
    // data-parallel baseline also gains from eight waves, held the per-shape
    // Stream-K / data-parallel ratio 1 % higher but cost 1.4 % of the sweep's
    // time (0.9 % on a sweep drawn with another seed).
    if (cand[1] && cand[2]) {
        delete cand[1];
        cand[1] = nullptr;
    }
    // smallest estimate; between plans the HBM bound makes equal, the smaller
    // compute-model time
    skgemm_plan_s* best = nullptr;
    double best_t = 0.0, best_c = 0.0;
    for (skgemm_plan_s* c : cand) {
        if (!c) continue;
        double tc = 0.0;
        const double t = plan_estimate(c, &tc);
        if (!best || t < best_t || (t == best_t && tc < best_c)) {
            delete best;
            best = c;
            best_t = t;
            best_c = tc;
        } else {
            delete c;
        }
    }
    if (!best) return last;
    // An automatic single-GEMM plan that splits the small 16-bit tile's tiles
    // over more workgroups than CUs (two on some CUs) is replaced by a plan
    // of at most one workgroup per CU on the three-stage kernel where that
    // was measured faster: with at most half as many tiles as CUs, the
    // largest split that fits (floor(CUs / t) shares per tile; 56 of 70 BF16
    // sweep shapes with 12 or more iterations per tile, 6 % less time, warm
    // and cold); with more, data-parallel tiles where the tiles have fewer
    // than 32 iterations (33 of 41 shapes, 4-7 % less; with longer tiles the
    // split's two workgroups per CU win).  The grid-size model does not see
    // this: its constants come from problems small enough to stay in cache,
    // where the two kernels' iterations cost the same.
    // (the small tile's GEMM variants 1 and 2 take variant 8; its
    // convolution variant 4 takes variant 9)
    const int deep = best->variant == 4 ? kVariantDeepConv : best->variant == 1 || best->variant == 2 ? kVariantDeep : -1;
    const bool deep_ok = deep >= 0 && (o.tile_waves == 0 || o.tile_waves == 8) && best->occ > 0 &&
                         kernel_exists(best->dtype, best->akc, best->bkc, deep);
    if (deep_ok && !best->G && o.policy == SKGEMM_POLICY_AUTO && o.force_g == 0 &&
        best->policy == SKGEMM_POLICY_SK) {
        const int cus = best->p / best->occ;
        if (best->g_sk > cus && best->t <= cus) {
            skgemm_options_t od = o;
            bool take = false;
            if (2 * best->t <= cus && best->ipt >= 12) {
                od.policy = SKGEMM_POLICY_SK;
                od.force_g = (cus / best->t) * best->t;
                take = true;
            } else if (2 * best->t > cus && best->ipt < 32) {
                od.policy = SKGEMM_POLICY_DP;
                take = true;
            }
            if (take) {
                skgemm_status_t st = SKGEMM_OK;
                skgemm_plan_s* d = build_variant(base, deep, od, G, M, N, K, &st);
                if (!d && st == SKGEMM_ERR_HIP) {
                    delete best;
                    return st;
                }
                if (d && d->grid <= cus) {
                    delete best;
                    best = d;
                } else {
                    delete d;
                }
            }
        }
    }
    // A small-tile plan whose grid fits one workgroup per CU runs the
    // eight-wave tile on three LDS stages instead: same tile, schedule and
    // workspace, two k-slabs in flight instead of one.  A lone workgroup on
    // its CU waits on load latency in the two-stage pipeline; measured on
    // one-wave data-parallel problems (BF16, 256 tiles of 128x128) the
    // three-stage kernel runs 9-18 % faster than either two-stage layout,
    // and loses where tiles outnumber CUs (its 96 KiB of LDS allow one
    // workgroup per CU).  Not where the options ask for four waves.  The plan
    // keeps the model constants it was resolved with (the grid fits the new
    // capacity, so every choice the model made stands).
    if (deep_ok && best->variant != deep && best->grid > 0) {
        const int cus = best->p / best->occ;
        int occ = 1;            // its LDS leaves room for one workgroup per CU
        if (o.occupancy == 0) {
            int qc = 0, qo = 0;
            if (device_capacity(best->dtype, best->akc, best->bkc, deep, &qc, &qo) != SKGEMM_OK) qo = 0;
            occ = qo;
        }
        if (occ >= 1 && best->grid <= cus) {
            best->variant = deep;
            best->occ = occ;
            best->p = cus * occ;
        }
    }
    *out = best;
    return SKGEMM_OK;
}

// Appends one problem (shape as given) to the plan's iteration space.
static void add_problem(skgemm_plan_s* pl, int64_t M, int64_t N, int64_t K) {
    const int32_t Ml = int32_t(pl->swapped ? N : M), Nl = int32_t(pl->swapped ? M : N);
    const int64_t tm = cdiv(Ml, pl->BM), tn = cdiv(Nl, pl->BN), ipt = cdiv(K, pl->BK);
    if (pl->tile_base.empty()) {
        pl->tile_base.push_back(0);
        pl->iter_base.push_back(0);
    }
    pl->gM.push_back(M); pl->gN.push_back(N); pl->gK.push_back(K);
    pl->pM.push_back(Ml); pl->pN.push_back(Nl); pl->pK.push_back(int32_t(K));
    pl->ptm.push_back(int32_t(tm)); pl->ptn.push_back(int32_t(tn)); pl->pipt.push_back(int32_t(ipt));
    const int64_t tb = pl->tile_base.back() + tm * tn;
    pl->tile_base.push_back(int32_t(std::min<int64_t>(tb, kMaxDim)));
    pl->iter_base.push_back(pl->iter_base.back() + tm * tn * ipt);
}

// Operand re-layout (single GEMMs only).  A line of an operand is a row of its
// contiguous dimension: the M (or N) rows of a K-contiguous operand, the K
// rows of an MN-contiguous one.  When the lines as the caller is expected to
// pass them (leading dimension = line length) do not start on 128-byte
// boundaries, every 128-byte segment of a slab row spans two cache lines and
// moves from L2 twice (BF16 on MI355X, operands in 64-element-padded storage
// against the natural leading dimensions: 9-38 % of the GEMM's time).  A copy
// into 128-byte lines costs a second launch and a pass over the operand, so
// it pays only where the operand is read many times over: each of the
// other operand's tile panels (tile columns for A, tile rows for B) reads
// the whole operand once, so the misaligned bytes moved grow with
// MB x panels, while the copy moves about 2 MB.  Over the 183 ragged shapes of
// the BF16 sweep with at least 4 GFLOP, timed with no copy, A, B and both
// copied, the gain fits (us) 0.0288 MB.panels - 0.339 MB for a K-contiguous
// operand and 0.0205 MB.panels - 0.346 MB for an MN-contiguous one (the MB
// terms are the copy at about 6 TB/s); copying where the fit exceeds 6 us
// saved 2.4 % of those shapes' time in five-fold cross-validation and lost at
// most 7 % on a shape, against 4.8 % for the best choice per shape and a
// 13 % loss for always copying.
constexpr double kPackKcR = 0.0288, kPackKcMb = 0.339;
constexpr double kPackMnR = 0.0205, kPackMnMb = 0.346;
constexpr double kPackMarginUs = 6.0;
constexpr int64_t kPackMaxBytes = int64_t(1) << 31;

static void plan_packing(skgemm_plan_s* pl, int32_t relayout) {
    const int eb = elem_bytes(pl->ta);
    // after the fix-up part and never over the error word and flag area, which
    // every plan sharing a workspace keeps at the same place and expects zero
    size_t off = (std::max(pl->ws_bytes, pl->partials_off) + 255) & ~size_t(255);
    for (int x = 0; x < 2; ++x) {
        const bool kc = x == 0 ? pl->akc : pl->bkc;
        const int64_t outer = x == 0 ? pl->Ml : pl->Nl;
        const int64_t lines = kc ? outer : pl->K, cols = kc ? pl->K : outer;
        const int64_t align = 128 / eb;
        pl->pack_lines[x] = lines;
        pl->pack_cols[x] = cols;
        pl->pack_ld[x] = (cols + align - 1) / align * align;
        const int64_t bytes = lines * pl->pack_ld[x] * eb;
        const double mb = double(lines) * double(cols) * eb / 1e6;
        // panels of the other operand, each of which reads this one whole
        const double panels = double(x == 0 ? cdiv(pl->Nl, pl->BN) : cdiv(pl->Ml, pl->BM));
        const double gain = kc ? kPackKcR * mb * panels - kPackKcMb * mb : kPackMnR * mb * panels - kPackMnMb * mb;
        // relayout masks name the caller's A and B; x is the launched operand
        const int caller = pl->swapped ? 1 - x : x;
        const bool wanted = relayout == 0 ? gain > kPackMarginUs : relayout > 0 && ((relayout >> caller) & 1);
        pl->pack[x] = lines > 0 && cols > 0 && (cols * eb) % 128 != 0 && bytes <= kPackMaxBytes &&
                      pl->pack_ld[x] <= kMaxDim && wanted;
        if (pl->pack[x]) {
            pl->pack_off[x] = off;
            off += (size_t(bytes) + 255) & ~size_t(255);
        }
    }
    pl->ws_total = (pl->pack[0] || pl->pack[1]) ? off : pl->ws_bytes;
}

// SKGEMM_LOG=1 in the environment: one line on stderr per plan built, with
// the decision (launch kind, shape, tile, resolved policy and grid, modelled
// time).  Read once per process.
static void log_plan(const skgemm_plan_s* pl) {
    static const bool on = [] {
        const char* v = std::getenv("SKGEMM_LOG");
        return v && v[0] && !(v[0] == '0' && !v[1]);
    }();
    if (!on) return;
    static const char* const kPol[] = {"auto", "dp", "sk", "dp_1tile_sk", "2tile_sk_dp", "paper"};
    const char* kind = pl->conv ? "conv" : pl->G ? "grouped" : pl->batch > 1 ? "batched" : "gemm";
    const double est = plan_estimate(pl, nullptr);
    std::fprintf(stderr,
                 "skgemm: plan %s M=%lld N=%lld K=%lld G=%d batch=%lld dtype=%d tile=%dx%dx%d/%d policy=%s "
                 "tiles=%d ipt=%d sk_tiles=%d g_sk=%d grid=%d p=%d est_us=%.2f pack=%d%d stages=%d\n",
                 kind, (long long)pl->M, (long long)pl->N, (long long)pl->K, pl->G, (long long)pl->batch, pl->dtype,
                 pl->BM, pl->BN, pl->BK, kernel_threads(pl->dtype, pl->variant) / 64,
                 pl->policy >= 0 && pl->policy <= 5 ? kPol[pl->policy] : "?", pl->t, pl->ipt, pl->sk_tiles,
                 pl->g_sk, pl->grid, pl->p, est, pl->pack[0] ? 1 : 0, pl->pack[1] ? 1 : 0,
                 tile_for(pl->dtype, pl->variant).ns);
}

skgemm_status_t skgemm_plan(skgemm_plan_t* out, int64_t M, int64_t N, int64_t K, skgemm_layout_t la,
                            skgemm_layout_t lb, skgemm_layout_t lc, skgemm_dtype_t ta, skgemm_dtype_t tb,
                            skgemm_dtype_t tc, const skgemm_options_t* opt) {
    if (!out) return SKGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (M < 0 || N < 0 || K < 0 || M > kMaxDim || N > kMaxDim || K > kMaxDim) return SKGEMM_ERR_INVALID_ARG;
    skgemm_options_t o;
    skgemm_default_options(&o);
    if (opt) o = *opt;
    if (o.hybrid_min_waves <= 0) o.hybrid_min_waves = 2;
    skgemm_plan_s base{};
    skgemm_status_t st = init_common(&base, la, lb, lc, ta, tb, tc, o);
    if (st != SKGEMM_OK) return st;
    base.M = M; base.N = N; base.K = K;
    base.G = 0;
    base.batch = 1;
    base.conv = false;
    base.order.assign(1, 0);
    skgemm_plan_s* pl = nullptr;
    st = plan_variants(&base, o, 1, &M, &N, &K, &pl);
    if (st != SKGEMM_OK) return st;
    plan_packing(pl, o.relayout);
    log_plan(pl);
    *out = pl;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_conv_plan(skgemm_plan_t* out, const skgemm_conv_t* cv, skgemm_dtype_t t_in,
                                 skgemm_dtype_t t_out, const skgemm_options_t* opt) {
    if (!out || !cv) return SKGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    const skgemm_conv_t& c = *cv;
    if (c.n < 0 || c.h < 1 || c.w < 1 || c.c < 1 || c.k < 0 || c.r < 1 || c.s < 1 || c.pad_h < 0 || c.pad_w < 0 ||
        c.stride_h < 1 || c.stride_w < 1 || c.dil_h < 1 || c.dil_w < 1)
        return SKGEMM_ERR_INVALID_ARG;
    const int64_t P = (int64_t(c.h) + 2 * c.pad_h - int64_t(c.dil_h) * (c.r - 1) - 1) / c.stride_h + 1;
    const int64_t Q = (int64_t(c.w) + 2 * c.pad_w - int64_t(c.dil_w) * (c.s - 1) - 1) / c.stride_w + 1;
    if (int64_t(c.h) + 2 * c.pad_h < int64_t(c.dil_h) * (c.r - 1) + 1 ||
        int64_t(c.w) + 2 * c.pad_w < int64_t(c.dil_w) * (c.s - 1) + 1)
        return SKGEMM_ERR_INVALID_ARG;                     // the window does not fit the padded image
    if (t_in != SKGEMM_BF16 && t_in != SKGEMM_F16) return SKGEMM_ERR_UNSUPPORTED;
    // whole k-slabs of channels (one filter tap per slab) and 32-bit gather offsets
    if (c.c % kTile16.bk != 0) return SKGEMM_ERR_UNSUPPORTED;
    const int64_t in_bytes = int64_t(c.n) * c.h * c.w * c.c * elem_bytes(t_in);
    if (in_bytes > kMaxDim) return SKGEMM_ERR_UNSUPPORTED;
    const int64_t M = int64_t(c.n) * P * Q, N = c.k, K = int64_t(c.r) * c.s * c.c;
    if (M > kMaxDim || K > kMaxDim) return SKGEMM_ERR_UNSUPPORTED;
    skgemm_options_t o;
    skgemm_default_options(&o);
    if (opt) o = *opt;
    if (o.hybrid_min_waves <= 0) o.hybrid_min_waves = 2;
    skgemm_plan_s base{};
    // the GEMM view: A (gathered) K-contiguous, the filters a column-major B, C row-major
    skgemm_status_t st = init_common(&base, SKGEMM_ROW_MAJOR, SKGEMM_COL_MAJOR, SKGEMM_ROW_MAJOR, t_in, t_in, t_out, o);
    if (st != SKGEMM_OK) return st;
    base.M = M; base.N = N; base.K = K;
    base.G = 0;
    base.batch = 1;
    base.conv = true;
    base.cv = ConvArgs{int32_t(c.n), int32_t(c.h), int32_t(c.w), int32_t(c.c), int32_t(P), int32_t(Q), int32_t(c.r),
                       int32_t(c.s), int32_t(c.pad_h), int32_t(c.pad_w), int32_t(c.stride_h), int32_t(c.stride_w),
                       int32_t(c.dil_h), int32_t(c.dil_w)};
    base.order.assign(1, 0);
    skgemm_plan_s* pl = nullptr;
    st = plan_variants(&base, o, 1, &base.M, &base.N, &base.K, &pl);
    if (st != SKGEMM_OK) return st;
    log_plan(pl);
    *out = pl;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_grouped_plan(skgemm_plan_t* out, int32_t G, const int64_t* M, const int64_t* N,
                                    const int64_t* K, skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc,
                                    skgemm_dtype_t ta, skgemm_dtype_t tb, skgemm_dtype_t tc,
                                    const skgemm_options_t* opt) {
    if (!out) return SKGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (G <= 0 || G > (1 << 20) || !M || !N || !K) return SKGEMM_ERR_INVALID_ARG;
    for (int i = 0; i < G; ++i) {
        if (M[i] < 0 || N[i] < 0 || K[i] < 0 || M[i] > kMaxDim || N[i] > kMaxDim || K[i] > kMaxDim)
            return SKGEMM_ERR_INVALID_ARG;
    }
    skgemm_options_t o;
    skgemm_default_options(&o);
    if (opt) o = *opt;
    if (o.hybrid_min_waves <= 0) o.hybrid_min_waves = 2;
    skgemm_plan_s base{};
    skgemm_status_t st = init_common(&base, la, lb, lc, ta, tb, tc, o);
    if (st != SKGEMM_OK) return st;
    base.G = G;
    base.batch = 1;
    base.conv = false;
    // iteration-space order: problems with MAC-loop iterations in the given
    // order, then the K = 0 problems that have tiles (epilogue only)
    base.order.clear();
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < G; ++i)
            if ((K[i] == 0 && M[i] > 0 && N[i] > 0) == (pass == 1)) base.order.push_back(i);
    base.M = base.N = base.K = 0;
    base.Ml = base.Nl = base.Kl = 0;
    base.tm = base.tn = base.ipt = 0;
    skgemm_plan_s* pl = nullptr;
    st = plan_variants(&base, o, G, M, N, K, &pl);
    if (st != SKGEMM_OK) return st;
    log_plan(pl);
    *out = pl;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_workspace_size(skgemm_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return SKGEMM_ERR_INVALID_ARG;
    *bytes = plan->ws_total;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_trace_capacity(skgemm_plan_t plan, size_t* n_records) {
    if (!plan || !n_records) return SKGEMM_ERR_INVALID_ARG;
    *n_records = size_t(plan->grid) * size_t(plan->max_segs);
    return SKGEMM_OK;
}

// Leading-dimension, pointer and 32-bit offset checks for one problem as
// given; fills the launched operand fields of e.
static skgemm_status_t check_problem(const skgemm_plan_s* pl, int64_t M, int64_t N, int64_t K, const void* A,
                                     int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, GroupEntry* e) {
    const int64_t a_min = pl->la == SKGEMM_ROW_MAJOR ? K : M;
    const int64_t b_min = pl->lb == SKGEMM_ROW_MAJOR ? N : K;
    const int64_t c_min = pl->lc == SKGEMM_ROW_MAJOR ? N : M;
    if (lda < std::max<int64_t>(1, a_min) || ldb < std::max<int64_t>(1, b_min) || ldc < std::max<int64_t>(1, c_min))
        return SKGEMM_ERR_INVALID_ARG;
    if (M > 0 && N > 0) {
        if (!C) return SKGEMM_ERR_INVALID_ARG;
        if (K > 0 && (!A || !B)) return SKGEMM_ERR_INVALID_ARG;
    }
    const int eb = elem_bytes(pl->ta);
    e->A = pl->swapped ? B : A;
    e->B = pl->swapped ? A : B;
    e->lda = pl->swapped ? ldb : lda;
    e->ldb = pl->swapped ? lda : ldb;
    e->C = C;
    e->ldc = ldc;
    // Loads use 32-bit offsets within one tile's slab of each operand.
    const int64_t lim = (int64_t(1) << 31) - 1;
    const int64_t span_a = pl->akc ? int64_t(pl->BM) * e->lda * eb + 128 : int64_t(pl->BK) * e->lda * eb + 512;
    const int64_t span_b = pl->bkc ? int64_t(pl->BN) * e->ldb * eb + 128 : int64_t(pl->BK) * e->ldb * eb + 512;
    if (span_a > lim || span_b > lim) return SKGEMM_ERR_UNSUPPORTED;
    return SKGEMM_OK;
}

static void fill_schedule_args(const skgemm_plan_s* pl, KArgs* a, void* workspace, int32_t* trace,
                               uint64_t* times) {
    a->t = pl->t;
    a->sk_tiles = pl->sk_tiles; a->g_sk = pl->g_sk;
    a->sk_iters = int32_t(pl->sk_iters);
    a->sk_q = pl->sk_q; a->sk_r = pl->sk_r;
    a->grid = pl->grid;
    a->sk_first = pl->sk_first ? 1 : 0;
    a->dp_only = pl->g_sk == 0 ? 1 : 0;
    a->out_dtype = pl->out;
    a->vec_a = 16;
    a->vec_b = 16;
    if (pl->ws_bytes) {
        unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
        a->err = reinterpret_cast<int32_t*>(ws);
        a->flags = reinterpret_cast<int32_t*>(ws + pl->flags_off);
        a->partials = reinterpret_cast<float*>(ws + pl->partials_off);
    }
    a->trace = trace;
    a->times = trace ? times : nullptr;
    a->trace_per_wg = trace ? pl->max_segs : 0;
    a->spin_limit = pl->spin_limit;
    a->sk_prop = pl->share_prop ? 1 : 0;
    a->raster = pl->raster;
    a->xcds = pl->xcds;
    a->coop_s = pl->coop_s;
    a->batch = int32_t(pl->batch);
    a->t1 = pl->tm * pl->tn;
    if (pl->conv) a->conv = pl->cv;
}

static skgemm_status_t run_impl(skgemm_plan_t pl, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                                int64_t ldc, float alpha, float beta, const float* scale_a, const float* scale_b,
                                void* workspace, size_t ws_bytes, int32_t* trace, uint64_t* times,
                                size_t trace_records, hipStream_t stream, const int64_t* strides = nullptr) {
    if (!pl || pl->G || pl->conv) return SKGEMM_ERR_INVALID_ARG;
    if ((pl->batch > 1) != (strides != nullptr)) return SKGEMM_ERR_INVALID_ARG;
    GroupEntry e;
    std::memset(&e, 0, sizeof(e));
    skgemm_status_t st = check_problem(pl, pl->M, pl->N, pl->K, A, lda, B, ldb, C, ldc, &e);
    if (st != SKGEMM_OK) return st;
    if (pl->M == 0 || pl->N == 0) return SKGEMM_OK;
    if (pl->ws_bytes) {
        if (!workspace || ws_bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255))
            return SKGEMM_ERR_WORKSPACE;
    }
    if (trace && trace_records < size_t(pl->grid) * size_t(pl->max_segs)) return SKGEMM_ERR_INVALID_ARG;
    // re-layout of operands whose lines, as passed, are not 128-byte aligned
    // (only with a workspace of the plan's full size: a smaller one that
    // still holds the fix-up runs the GEMM on the operands as given)
    if ((pl->pack[0] || pl->pack[1]) && workspace && ws_bytes >= pl->ws_total &&
        !(reinterpret_cast<uintptr_t>(workspace) & 255)) {
        const int eb = elem_bytes(pl->ta);
        for (int x = 0; x < 2; ++x) {
            const void*& op = x == 0 ? e.A : e.B;
            int64_t& ld = x == 0 ? e.lda : e.ldb;
            if (!pl->pack[x] || (ld * eb) % 128 == 0) continue;
            // the copy's leading dimension must keep a tile's slab within 32-bit offsets
            const bool kc = x == 0 ? pl->akc : pl->bkc;
            const int64_t span = kc ? int64_t(x == 0 ? pl->BM : pl->BN) * pl->pack_ld[x] * eb + 128
                                    : int64_t(pl->BK) * pl->pack_ld[x] * eb + 512;
            if (span > kMaxDim) continue;
            void* dst = static_cast<unsigned char*>(workspace) + pl->pack_off[x];
            const int rc = launch_pack(op, ld, pl->pack_lines[x], pl->pack_cols[x], dst, pl->pack_ld[x], eb, stream);
            if (rc != int(hipSuccess)) return SKGEMM_ERR_HIP;
            op = dst;
            ld = pl->pack_ld[x];
        }
    }
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = e.A; a.B = e.B; a.C = e.C;
    a.lda = e.lda; a.ldb = e.ldb; a.ldc = e.ldc;
    a.scale_a = pl->swapped ? scale_b : scale_a;
    a.scale_b = pl->swapped ? scale_a : scale_b;
    a.M = pl->Ml; a.N = pl->Nl; a.K = pl->Kl;
    a.tm = pl->tm; a.tn = pl->tn; a.ipt = pl->ipt;
    a.alpha = alpha;
    a.beta = beta;
    fill_schedule_args(pl, &a, workspace, trace, times);
    if (strides) {
        const int64_t eb = elem_bytes(pl->ta), ec = elem_bytes(pl->tc);
        a.stride_a = (pl->swapped ? strides[1] : strides[0]) * eb;
        a.stride_b = (pl->swapped ? strides[0] : strides[1]) * eb;
        a.stride_c = strides[2] * ec;
    }
    if (pl->grid == 0) return SKGEMM_OK;
    const int rc = launch_gemm(pl->dtype, pl->akc, pl->bkc, pl->variant, a, pl->grid, stream);
    return rc == int(hipSuccess) ? SKGEMM_OK : SKGEMM_ERR_HIP;
}

skgemm_status_t skgemm_run(skgemm_plan_t plan, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                           int64_t ldc, float alpha, float beta, const float* scale_a, const float* scale_b,
                           void* workspace, size_t ws_bytes, hipStream_t stream) {
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, nullptr,
                    nullptr, 0, stream);
}

skgemm_status_t skgemm_run_traced(skgemm_plan_t plan, const void* A, int64_t lda, const void* B, int64_t ldb,
                                  void* C, int64_t ldc, float alpha, float beta, const float* scale_a,
                                  const float* scale_b, void* workspace, size_t ws_bytes, int32_t* trace,
                                  size_t trace_records, hipStream_t stream) {
    if (!trace) return SKGEMM_ERR_INVALID_ARG;
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, trace,
                    nullptr, trace_records, stream);
}

skgemm_status_t skgemm_run_timed(skgemm_plan_t plan, const void* A, int64_t lda, const void* B, int64_t ldb,
                                 void* C, int64_t ldc, float alpha, float beta, const float* scale_a,
                                 const float* scale_b, void* workspace, size_t ws_bytes, int32_t* trace,
                                 uint64_t* times, size_t trace_records, hipStream_t stream) {
    if (!trace || !times) return SKGEMM_ERR_INVALID_ARG;
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, trace,
                    times, trace_records, stream);
}

skgemm_status_t skgemm_realtime_hz(int64_t* hz) {
    if (!hz) return SKGEMM_ERR_INVALID_ARG;
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        return SKGEMM_ERR_HIP;
    *hz = int64_t(khz) * 1000;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_batched_plan(skgemm_plan_t* out, int64_t batch, int64_t M, int64_t N, int64_t K,
                                    skgemm_layout_t la, skgemm_layout_t lb, skgemm_layout_t lc, skgemm_dtype_t ta,
                                    skgemm_dtype_t tb, skgemm_dtype_t tc, const skgemm_options_t* opt) {
    if (!out) return SKGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (batch < 1 || batch > kMaxDim || M < 0 || N < 0 || K < 0 || M > kMaxDim || N > kMaxDim || K > kMaxDim)
        return SKGEMM_ERR_INVALID_ARG;
    skgemm_options_t o;
    skgemm_default_options(&o);
    if (opt) o = *opt;
    if (o.hybrid_min_waves <= 0) o.hybrid_min_waves = 2;
    skgemm_plan_s base{};
    skgemm_status_t st = init_common(&base, la, lb, lc, ta, tb, tc, o);
    if (st != SKGEMM_OK) return st;
    base.M = M; base.N = N; base.K = K;
    base.G = 0;
    base.batch = batch;
    base.conv = false;
    base.order.assign(1, 0);
    skgemm_plan_s* pl = nullptr;
    st = plan_variants(&base, o, 1, &M, &N, &K, &pl);
    if (st != SKGEMM_OK) return st;
    log_plan(pl);
    *out = pl;
    return SKGEMM_OK;
}

static skgemm_status_t batched_impl(skgemm_plan_t plan, const void* A, int64_t lda, int64_t stride_a, const void* B,
                                    int64_t ldb, int64_t stride_b, void* C, int64_t ldc, int64_t stride_c,
                                    float alpha, float beta, const float* scale_a, const float* scale_b,
                                    void* workspace, size_t ws_bytes, int32_t* trace, size_t trace_records,
                                    hipStream_t stream) {
    if (!plan || plan->G || plan->batch < 1) return SKGEMM_ERR_INVALID_ARG;
    if (stride_a < 0 || stride_b < 0 || stride_c < 0) return SKGEMM_ERR_INVALID_ARG;
    // consecutive C matrices must not overlap (each problem writes its whole C)
    const int64_t c_extent = plan->lc == SKGEMM_ROW_MAJOR ? (plan->M - 1) * ldc + plan->N : (plan->N - 1) * ldc + plan->M;
    if (plan->batch > 1 && plan->M > 0 && plan->N > 0 && stride_c < c_extent) return SKGEMM_ERR_INVALID_ARG;
    if (plan->batch == 1)
        return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, trace,
                        nullptr, trace_records, stream);
    const int64_t strides[3] = {stride_a, stride_b, stride_c};
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, trace,
                    nullptr, trace_records, stream, strides);
}

skgemm_status_t skgemm_batched_run(skgemm_plan_t plan, const void* A, int64_t lda, int64_t stride_a, const void* B,
                                   int64_t ldb, int64_t stride_b, void* C, int64_t ldc, int64_t stride_c, float alpha,
                                   float beta, const float* scale_a, const float* scale_b, void* workspace,
                                   size_t ws_bytes, hipStream_t stream) {
    return batched_impl(plan, A, lda, stride_a, B, ldb, stride_b, C, ldc, stride_c, alpha, beta, scale_a, scale_b,
                        workspace, ws_bytes, nullptr, 0, stream);
}

skgemm_status_t skgemm_batched_run_traced(skgemm_plan_t plan, const void* A, int64_t lda, int64_t stride_a,
                                          const void* B, int64_t ldb, int64_t stride_b, void* C, int64_t ldc,
                                          int64_t stride_c, float alpha, float beta, const float* scale_a,
                                          const float* scale_b, void* workspace, size_t ws_bytes, int32_t* trace,
                                          size_t trace_records, hipStream_t stream) {
    if (!trace) return SKGEMM_ERR_INVALID_ARG;
    return batched_impl(plan, A, lda, stride_a, B, ldb, stride_b, C, ldc, stride_c, alpha, beta, scale_a, scale_b,
                        workspace, ws_bytes, trace, trace_records, stream);
}

static skgemm_status_t conv_impl(skgemm_plan_t pl, const void* x, const void* w, void* y, float alpha, float beta,
                                 void* workspace, size_t ws_bytes, int32_t* trace, size_t trace_records,
                                 hipStream_t stream) {
    if (!pl || !pl->conv) return SKGEMM_ERR_INVALID_ARG;
    if (pl->M == 0 || pl->N == 0) return SKGEMM_OK;
    if (!y || !x || !w) return SKGEMM_ERR_INVALID_ARG;
    if (pl->ws_bytes) {
        if (!workspace || ws_bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255))
            return SKGEMM_ERR_WORKSPACE;
    }
    if (trace && trace_records < size_t(pl->grid) * size_t(pl->max_segs)) return SKGEMM_ERR_INVALID_ARG;
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.A = x; a.B = w; a.C = y;
    a.lda = pl->K; a.ldb = pl->K; a.ldc = pl->N;
    a.M = pl->Ml; a.N = pl->Nl; a.K = pl->Kl;
    a.tm = pl->tm; a.tn = pl->tn; a.ipt = pl->ipt;
    a.alpha = alpha;
    a.beta = beta;
    fill_schedule_args(pl, &a, workspace, trace, nullptr);
    if (pl->grid == 0) return SKGEMM_OK;
    const int rc = launch_gemm(pl->dtype, pl->akc, pl->bkc, pl->variant, a, pl->grid, stream);
    return rc == int(hipSuccess) ? SKGEMM_OK : SKGEMM_ERR_HIP;
}

skgemm_status_t skgemm_conv_run(skgemm_plan_t plan, const void* x, const void* w, void* y, float alpha, float beta,
                                void* workspace, size_t ws_bytes, hipStream_t stream) {
    return conv_impl(plan, x, w, y, alpha, beta, workspace, ws_bytes, nullptr, 0, stream);
}

skgemm_status_t skgemm_conv_run_traced(skgemm_plan_t plan, const void* x, const void* w, void* y, float alpha,
                                       float beta, void* workspace, size_t ws_bytes, int32_t* trace,
                                       size_t trace_records, hipStream_t stream) {
    if (!trace) return SKGEMM_ERR_INVALID_ARG;
    return conv_impl(plan, x, w, y, alpha, beta, workspace, ws_bytes, trace, trace_records, stream);
}

skgemm_status_t skgemm_grouped_table_size(skgemm_plan_t pl, size_t* bytes) {
    if (!pl || !bytes || !pl->G) return SKGEMM_ERR_INVALID_ARG;
    *bytes = size_t(pl->G) * sizeof(GroupEntry);
    return SKGEMM_OK;
}

skgemm_status_t skgemm_grouped_table(skgemm_plan_t pl, const skgemm_group_args_t* args, void* table,
                                     size_t bytes) {
    if (!pl || !pl->G || !args || !table || bytes < size_t(pl->G) * sizeof(GroupEntry)) return SKGEMM_ERR_INVALID_ARG;
    GroupEntry* out = reinterpret_cast<GroupEntry*>(table);
    for (int i = 0; i < pl->G; ++i) {
        GroupEntry e;
        std::memset(&e, 0, sizeof(e));
        const skgemm_group_args_t& g = args[pl->order[i]];
        const skgemm_status_t st =
            check_problem(pl, pl->gM[i], pl->gN[i], pl->gK[i], g.A, g.lda, g.B, g.ldb, g.C, g.ldc, &e);
        if (st != SKGEMM_OK) return st;
        e.iter_base = pl->iter_base[i];
        e.M = pl->pM[i]; e.N = pl->pN[i]; e.K = pl->pK[i];
        e.tm = pl->ptm[i]; e.tn = pl->ptn[i]; e.ipt = pl->pipt[i];
        e.tile_base = pl->tile_base[i];
        e.alpha = g.alpha;
        e.beta = g.beta;
        std::memcpy(&out[i], &e, sizeof(e));
    }
    return SKGEMM_OK;
}

static skgemm_status_t grouped_impl(skgemm_plan_t pl, const void* table_dev, void* workspace, size_t ws_bytes,
                                    int32_t* trace, size_t trace_records, hipStream_t stream) {
    if (!pl || !pl->G || !table_dev) return SKGEMM_ERR_INVALID_ARG;
    if (pl->ws_bytes) {
        if (!workspace || ws_bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255))
            return SKGEMM_ERR_WORKSPACE;
    }
    if (trace && trace_records < size_t(pl->grid) * size_t(pl->max_segs)) return SKGEMM_ERR_INVALID_ARG;
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.group = reinterpret_cast<const GroupEntry*>(table_dev);
    a.G = pl->G;
    fill_schedule_args(pl, &a, workspace, trace, nullptr);
    if (pl->grid == 0) return SKGEMM_OK;
    const int rc = launch_gemm(pl->dtype, pl->akc, pl->bkc, pl->variant, a, pl->grid, stream);
    return rc == int(hipSuccess) ? SKGEMM_OK : SKGEMM_ERR_HIP;
}

skgemm_status_t skgemm_grouped_run(skgemm_plan_t plan, const void* table_dev, void* workspace, size_t ws_bytes,
                                   hipStream_t stream) {
    return grouped_impl(plan, table_dev, workspace, ws_bytes, nullptr, 0, stream);
}

skgemm_status_t skgemm_grouped_run_traced(skgemm_plan_t plan, const void* table_dev, void* workspace,
                                          size_t ws_bytes, int32_t* trace, size_t trace_records,
                                          hipStream_t stream) {
    if (!trace) return SKGEMM_ERR_INVALID_ARG;
    return grouped_impl(plan, table_dev, workspace, ws_bytes, trace, trace_records, stream);
}

skgemm_status_t skgemm_plan_info(skgemm_plan_t pl, int64_t* info, int32_t n) {
    if (!pl || !info || n < 0) return SKGEMM_ERR_INVALID_ARG;
    const int64_t v[30] = {pl->Ml, pl->Nl, pl->Kl, pl->swapped ? 1 : 0, pl->BM, pl->BN, pl->BK, pl->tm, pl->tn,
                           pl->t, pl->ipt, pl->policy, pl->sk_tiles, pl->g_sk, pl->grid, pl->sk_first ? 1 : 0,
                           pl->p, pl->hybrid_min_waves, pl->akc ? 1 : 0, pl->bkc ? 1 : 0, pl->G,
                           pl->share_prop ? SKGEMM_SHARE_PROPORTIONAL : SKGEMM_SHARE_LEADING, pl->coop_s,
                           pl->occ, kernel_threads(pl->dtype, pl->variant) / 64, pl->batch,
                           pl->pack[0] ? 1 : 0, pl->pack[1] ? 1 : 0, int64_t(pl->ws_bytes),
                           tile_for(pl->dtype, pl->variant).ns};
    for (int i = 0; i < n && i < 30; ++i) info[i] = v[i];
    return SKGEMM_OK;
}

skgemm_status_t skgemm_model_constants(skgemm_plan_t pl, double* abcde) {
    if (!pl || !abcde) return SKGEMM_ERR_INVALID_ARG;
    for (int i = 0; i < 5; ++i) abcde[i] = pl->model[i];
    return SKGEMM_OK;
}

skgemm_status_t skgemm_schedule(skgemm_plan_t pl, int32_t* records, size_t cap, size_t* n) {
    if (!pl || !n) return SKGEMM_ERR_INVALID_ARG;
    size_t count = 0;
    for (int x = 0; x < pl->grid; ++x) {
        walk(*pl, x, [&](int seq, int tile, int lo, int hi, int role, int p0, int p1) {
            if (records && count < cap) {
                int32_t* r = records + count * kTraceFields;
                r[0] = x; r[1] = seq; r[2] = tile; r[3] = lo; r[4] = hi; r[5] = role; r[6] = p0; r[7] = p1;
            }
            ++count;
        });
    }
    *n = count;
    return (records && count > cap) ? SKGEMM_ERR_INVALID_ARG : SKGEMM_OK;
}

skgemm_status_t skgemm_check_device_error(const void* workspace, hipStream_t stream) {
    if (!workspace) return SKGEMM_ERR_INVALID_ARG;
    int32_t word = 0;
    if (hipMemcpyAsync(&word, workspace, sizeof(word), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return SKGEMM_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return SKGEMM_ERR_HIP;
    return word == 0 ? SKGEMM_OK : SKGEMM_ERR_TIMEOUT;
}

skgemm_status_t skgemm_quantize_workspace_size(size_t* bytes) {
    if (!bytes) return SKGEMM_ERR_INVALID_ARG;
    *bytes = size_t(quant_workspace_floats()) * sizeof(float);
    return SKGEMM_OK;
}

skgemm_status_t skgemm_quantize_e4m3(const void* X, skgemm_dtype_t tx, int64_t rows, int64_t cols,
                                     skgemm_layout_t lx, int64_t ldx, void* Q, skgemm_layout_t lq, int64_t ldq,
                                     float* scale, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (tx != SKGEMM_F32 && tx != SKGEMM_BF16 && tx != SKGEMM_F16) return SKGEMM_ERR_UNSUPPORTED;
    if (rows < 0 || cols < 0 || (lx != SKGEMM_ROW_MAJOR && lx != SKGEMM_COL_MAJOR) ||
        (lq != SKGEMM_ROW_MAJOR && lq != SKGEMM_COL_MAJOR))
        return SKGEMM_ERR_INVALID_ARG;
    const int64_t x_min = lx == SKGEMM_ROW_MAJOR ? cols : rows, q_min = lq == SKGEMM_ROW_MAJOR ? cols : rows;
    if (ldx < std::max<int64_t>(1, x_min) || ldq < std::max<int64_t>(1, q_min)) return SKGEMM_ERR_INVALID_ARG;
    if (!scale || (rows > 0 && cols > 0 && (!X || !Q))) return SKGEMM_ERR_INVALID_ARG;
    if ((rows + 63) / 64 > 65535 || (cols + 63) / 64 > kMaxDim) return SKGEMM_ERR_UNSUPPORTED;
    const size_t need = size_t(quant_workspace_floats()) * sizeof(float);
    if (!workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 3)) return SKGEMM_ERR_WORKSPACE;
    const int rc = launch_quantize(to_dt(tx), X, rows, cols, ldx, lx == SKGEMM_COL_MAJOR,
                                   reinterpret_cast<uint8_t*>(Q), ldq, lq == SKGEMM_COL_MAJOR, scale,
                                   reinterpret_cast<float*>(workspace), stream);
    return rc == int(hipSuccess) ? SKGEMM_OK : SKGEMM_ERR_HIP;
}

skgemm_status_t skgemm_plan_destroy(skgemm_plan_t plan) {
    delete plan;
    return SKGEMM_OK;
}

const char* skgemm_status_string(skgemm_status_t s) {
    switch (s) {
        case SKGEMM_OK: return "ok";
        case SKGEMM_ERR_INVALID_ARG: return "invalid argument";
        case SKGEMM_ERR_UNSUPPORTED: return "unsupported";
        case SKGEMM_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case SKGEMM_ERR_CAPACITY: return "grid exceeds co-resident workgroups";
        case SKGEMM_ERR_HIP: return "HIP runtime error";
        case SKGEMM_ERR_TIMEOUT: return "fix-up wait timed out on the device";
    }
    return "unknown status";
}

}  // extern "C"
