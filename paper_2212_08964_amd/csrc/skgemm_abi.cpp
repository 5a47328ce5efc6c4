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
#include <cstring>
#include <mutex>
#include <new>

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
    // tiling and schedule
    int BM, BN, BK;
    int tm, tn, t, ipt;
    int policy;
    int sk_tiles, g_sk, grid;
    bool sk_first;
    int p, hybrid_min_waves;
    int sk_q, sk_r;
    double model[4];
    // workspace layout
    size_t ws_bytes, flags_off, partials_off;
    int max_segs;
};

namespace {

int elem_bytes(skgemm_dtype_t t) {
    switch (t) {
        case SKGEMM_F32: return 4;
        case SKGEMM_F16:
        case SKGEMM_BF16: return 2;
        case SKGEMM_F8E4M3: return 1;
    }
    return 0;
}

int to_dt(skgemm_dtype_t t) {
    switch (t) {
        case SKGEMM_F32: return DT_F32;
        case SKGEMM_F16: return DT_F16;
        case SKGEMM_BF16: return DT_BF16;
        case SKGEMM_F8E4M3: return DT_F8;
    }
    return -1;
}

TileCfg tile_for(int dt) {
    switch (dt) {
        case DT_F32: return kTileF32;
        case DT_F8: return kTileF8;
        default: return kTile16;
    }
}

// Grid-size model constants (a, b, c, d) per input type, in units of one
// MAC-loop iteration (c = 1): a fixed per-workgroup cost, b the cost of
// publishing a partial tile, d the cost of adding one peer's partial.
void model_for(int dt, double* m) {
    switch (dt) {
        case DT_F32: m[0] = 3.0; m[1] = 1.0; m[2] = 1.0; m[3] = 1.0; break;
        case DT_F8: m[0] = 8.0; m[1] = 3.0; m[2] = 1.0; m[3] = 3.0; break;
        default: m[0] = 5.0; m[1] = 2.0; m[2] = 1.0; m[3] = 2.0; break;
    }
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

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

int share_start(int x, int q, int r) { return x * q + std::min(x, r); }

int owner_of(int i, int q, int r) { return (i < r * (q + 1)) ? i / (q + 1) : r + (i - r * (q + 1)) / q; }

// Walks the schedule of workgroup x exactly as the kernel does; calls
// emit(seq, tile, lo, hi, role, first_peer, last_peer) per segment.
template <class F>
int walk(const skgemm_plan_s& pl, int x, F&& emit) {
    int sk_it = 0, sk_end = 0;
    if (x < pl.g_sk) {
        sk_it = share_start(x, pl.sk_q, pl.sk_r);
        sk_end = share_start(x + 1, pl.sk_q, pl.sk_r);
    }
    int dp_tile = pl.sk_tiles + x;
    int seq = 0;
    for (;;) {
        const bool sk_left = sk_it < sk_end, dp_left = dp_tile < pl.t;
        if (!sk_left && !dp_left) break;
        const bool take_sk = pl.sk_first ? sk_left : !dp_left;
        int tile, lo, hi, role, p0 = -1, p1 = -1;
        if (take_sk) {
            tile = sk_it / pl.ipt;
            const int first = tile * pl.ipt, last = first + pl.ipt;
            lo = sk_it - first;
            hi = std::min(sk_end, last) - first;
            if (sk_it != first) {
                role = ROLE_PARTIAL;
            } else if (sk_end < last) {
                role = ROLE_OWNER;
                p0 = x + 1;
                p1 = owner_of(last - 1, pl.sk_q, pl.sk_r);
            } else {
                role = ROLE_FULL;
            }
            sk_it = last;
        } else {
            tile = dp_tile;
            lo = 0;
            hi = pl.ipt;
            role = ROLE_FULL;
            dp_tile += pl.grid;
        }
        emit(seq, tile, lo, hi, role, p0, p1);
        ++seq;
    }
    return seq;
}

struct DevInfo {
    int cus = 0;
    int occ[4][2][2] = {};
    bool have_occ[4][2][2] = {};
};
std::mutex g_dev_mu;
DevInfo g_dev[64];

skgemm_status_t device_capacity(int dt, bool akc, bool bkc, int* cus, int* occ) {
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
    if (!d.have_occ[dt][akc][bkc]) {
        const int o = kernel_occupancy(dt, akc, bkc);
        if (o <= 0) return SKGEMM_ERR_HIP;
        d.occ[dt][akc][bkc] = o;
        d.have_occ[dt][akc][bkc] = true;
    }
    *cus = d.cus;
    *occ = d.occ[dt][akc][bkc];
    return SKGEMM_OK;
}

constexpr int64_t kMaxDim = (int64_t(1) << 31) - 1;

}  // namespace

extern "C" {

void skgemm_default_options(skgemm_options_t* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->policy = SKGEMM_POLICY_AUTO;
    opt->hybrid_min_waves = 2;
}

skgemm_status_t skgemm_plan(skgemm_plan_t* out, int64_t M, int64_t N, int64_t K, skgemm_layout_t la,
                            skgemm_layout_t lb, skgemm_layout_t lc, skgemm_dtype_t ta, skgemm_dtype_t tb,
                            skgemm_dtype_t tc, const skgemm_options_t* opt) {
    if (!out) return SKGEMM_ERR_INVALID_ARG;
    *out = nullptr;
    if (M < 0 || N < 0 || K < 0 || M > kMaxDim || N > kMaxDim || K > kMaxDim) return SKGEMM_ERR_INVALID_ARG;
    if ((la != SKGEMM_ROW_MAJOR && la != SKGEMM_COL_MAJOR) || (lb != SKGEMM_ROW_MAJOR && lb != SKGEMM_COL_MAJOR) ||
        (lc != SKGEMM_ROW_MAJOR && lc != SKGEMM_COL_MAJOR))
        return SKGEMM_ERR_INVALID_ARG;
    if (to_dt(ta) < 0 || to_dt(tb) < 0 || to_dt(tc) < 0) return SKGEMM_ERR_INVALID_ARG;
    if (ta != tb) return SKGEMM_ERR_UNSUPPORTED;
    if (tc == SKGEMM_F8E4M3) return SKGEMM_ERR_UNSUPPORTED;
    if (ta != SKGEMM_F8E4M3 && ta != SKGEMM_F32 && tc != ta && tc != SKGEMM_F32) return SKGEMM_ERR_UNSUPPORTED;
    if (ta == SKGEMM_F32 && tc != SKGEMM_F32) return SKGEMM_ERR_UNSUPPORTED;
    skgemm_options_t o;
    skgemm_default_options(&o);
    if (opt) o = *opt;
    if (o.hybrid_min_waves <= 0) o.hybrid_min_waves = 2;
    if (o.force_g < 0 || o.num_cus < 0 || o.occupancy < 0) return SKGEMM_ERR_INVALID_ARG;
    if (o.policy < SKGEMM_POLICY_AUTO || o.policy > SKGEMM_POLICY_2TILE_SK_DP) return SKGEMM_ERR_INVALID_ARG;

    skgemm_plan_s* pl = new (std::nothrow) skgemm_plan_s();
    if (!pl) return SKGEMM_ERR_HIP;
    pl->M = M; pl->N = N; pl->K = K;
    pl->la = la; pl->lb = lb; pl->lc = lc;
    pl->ta = ta; pl->tc = tc;
    pl->dtype = to_dt(ta);
    pl->out = to_dt(tc);
    pl->swapped = (lc == SKGEMM_COL_MAJOR);
    const bool a_kc = (la == SKGEMM_ROW_MAJOR), b_kc = (lb == SKGEMM_COL_MAJOR);
    pl->Ml = int32_t(pl->swapped ? N : M);
    pl->Nl = int32_t(pl->swapped ? M : N);
    pl->Kl = int32_t(K);
    pl->akc = pl->swapped ? b_kc : a_kc;
    pl->bkc = pl->swapped ? a_kc : b_kc;
    if (!kernel_exists(pl->dtype, pl->akc, pl->bkc)) {
        delete pl;
        return SKGEMM_ERR_UNSUPPORTED;
    }
    const TileCfg tc_ = tile_for(pl->dtype);
    if ((o.tile_m && o.tile_m != tc_.bm) || (o.tile_n && o.tile_n != tc_.bn) || (o.tile_k && o.tile_k != tc_.bk)) {
        delete pl;
        return SKGEMM_ERR_UNSUPPORTED;
    }
    pl->BM = tc_.bm; pl->BN = tc_.bn; pl->BK = tc_.bk;
    model_for(pl->dtype, pl->model);
    pl->hybrid_min_waves = o.hybrid_min_waves;

    int cus = o.num_cus, occ = o.occupancy;
    if (cus == 0 || occ == 0) {
        int qc = 0, qo = 0;
        const skgemm_status_t st = device_capacity(pl->dtype, pl->akc, pl->bkc, &qc, &qo);
        if (st != SKGEMM_OK) {
            delete pl;
            return st;
        }
        if (cus == 0) cus = qc;
        if (occ == 0) occ = qo;
    }
    const int64_t p = int64_t(cus) * occ;
    if (p <= 0 || p > kMaxDim) {
        delete pl;
        return SKGEMM_ERR_INVALID_ARG;
    }
    pl->p = int(p);

    const int64_t tm = cdiv(pl->Ml, pl->BM), tn = cdiv(pl->Nl, pl->BN), ipt = cdiv(K, pl->BK);
    const int64_t t = tm * tn;
    if (t > kMaxDim || t * ipt > kMaxDim) {
        delete pl;
        return SKGEMM_ERR_UNSUPPORTED;
    }
    pl->tm = int(tm); pl->tn = int(tn); pl->t = int(t); pl->ipt = int(ipt);

    int policy = o.policy;
    pl->sk_tiles = 0; pl->g_sk = 0; pl->grid = 0; pl->sk_first = true;
    if (t > 0) {
        if (ipt == 0) policy = SKGEMM_POLICY_DP;
        const int64_t w = t / p, r = t % p;
        if (policy == SKGEMM_POLICY_AUTO) {
            if (r == 0) policy = SKGEMM_POLICY_DP;
            else if (w == 0) policy = SKGEMM_POLICY_SK;
            else if (w >= pl->hybrid_min_waves) policy = SKGEMM_POLICY_2TILE_SK_DP;
            else policy = SKGEMM_POLICY_DP_1TILE_SK;
        }
        if (policy == SKGEMM_POLICY_DP) {
            pl->grid = int(t);
        } else if (policy == SKGEMM_POLICY_SK) {
            pl->sk_tiles = int(t);
            if (o.force_g) pl->g_sk = o.force_g;
            else if (t >= p) pl->g_sk = int(p);
            else pl->g_sk = model_best_g(t, ipt, p, pl->model);
            pl->grid = pl->g_sk;
        } else {
            if (policy == SKGEMM_POLICY_DP_1TILE_SK) {
                pl->sk_tiles = int(r);
                pl->sk_first = false;
            } else {
                pl->sk_tiles = int(w == 0 ? t : r + p);
                pl->sk_first = true;
            }
            if (pl->sk_tiles) pl->g_sk = o.force_g ? o.force_g : int(std::min<int64_t>(p, pl->sk_tiles * ipt));
            pl->grid = (t - pl->sk_tiles > 0) ? int(p) : pl->g_sk;
            pl->grid = std::max(pl->grid, pl->g_sk);
        }
    }
    pl->policy = policy;
    // Owners wait on workgroups with higher indices, so every Stream-K
    // workgroup must be resident at once.
    if (pl->g_sk > pl->p) {
        delete pl;
        return SKGEMM_ERR_CAPACITY;
    }
    if (pl->g_sk) {
        const int64_t total = int64_t(pl->sk_tiles) * ipt;
        pl->sk_q = int(total / pl->g_sk);
        pl->sk_r = int(total % pl->g_sk);
    }
    pl->flags_off = kWsHeaderBytes;
    pl->partials_off = (kWsHeaderBytes + size_t(pl->g_sk) * kFlagStrideInts * 4 + 255) & ~size_t(255);
    pl->ws_bytes = pl->g_sk ? pl->partials_off + size_t(pl->g_sk) * pl->BM * pl->BN * 4 : 0;
    int mx = 0;
    for (int x = 0; x < pl->grid; ++x) mx = std::max(mx, walk(*pl, x, [](int, int, int, int, int, int, int) {}));
    pl->max_segs = mx;
    *out = pl;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_workspace_size(skgemm_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return SKGEMM_ERR_INVALID_ARG;
    *bytes = plan->ws_bytes;
    return SKGEMM_OK;
}

skgemm_status_t skgemm_trace_capacity(skgemm_plan_t plan, size_t* n_records) {
    if (!plan || !n_records) return SKGEMM_ERR_INVALID_ARG;
    *n_records = size_t(plan->grid) * size_t(plan->max_segs);
    return SKGEMM_OK;
}

static skgemm_status_t run_impl(skgemm_plan_t pl, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                                int64_t ldc, float alpha, float beta, const float* scale_a, const float* scale_b,
                                void* workspace, size_t ws_bytes, int32_t* trace, size_t trace_records,
                                hipStream_t stream) {
    if (!pl) return SKGEMM_ERR_INVALID_ARG;
    const int64_t M = pl->M, N = pl->N, K = pl->K;
    // leading dimensions follow each operand's own layout
    const int64_t a_min = pl->la == SKGEMM_ROW_MAJOR ? K : M;
    const int64_t b_min = pl->lb == SKGEMM_ROW_MAJOR ? N : K;
    const int64_t c_min = pl->lc == SKGEMM_ROW_MAJOR ? N : M;
    if (lda < std::max<int64_t>(1, a_min) || ldb < std::max<int64_t>(1, b_min) || ldc < std::max<int64_t>(1, c_min))
        return SKGEMM_ERR_INVALID_ARG;
    if (M == 0 || N == 0) return SKGEMM_OK;
    if (!C) return SKGEMM_ERR_INVALID_ARG;
    if (K > 0 && (!A || !B)) return SKGEMM_ERR_INVALID_ARG;
    if (pl->ws_bytes) {
        if (!workspace || ws_bytes < pl->ws_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255))
            return SKGEMM_ERR_WORKSPACE;
    }
    if (trace && trace_records < size_t(pl->grid) * size_t(pl->max_segs)) return SKGEMM_ERR_INVALID_ARG;

    KArgs a;
    std::memset(&a, 0, sizeof(a));
    const int eb = elem_bytes(pl->ta);
    a.A = pl->swapped ? B : A;
    a.B = pl->swapped ? A : B;
    a.lda = pl->swapped ? ldb : lda;
    a.ldb = pl->swapped ? lda : ldb;
    a.scale_a = pl->swapped ? scale_b : scale_a;
    a.scale_b = pl->swapped ? scale_a : scale_b;
    // Loads use 32-bit offsets within one tile's slab of each operand.
    const int64_t lim = (int64_t(1) << 31) - 1;
    const int64_t span_a = pl->akc ? int64_t(pl->BM) * a.lda * eb + 128 : int64_t(pl->BK) * a.lda * eb + 512;
    const int64_t span_b = pl->bkc ? int64_t(pl->BN) * a.ldb * eb + 128 : int64_t(pl->BK) * a.ldb * eb + 512;
    if (span_a > lim || span_b > lim) return SKGEMM_ERR_UNSUPPORTED;
    a.C = C;
    a.ldc = ldc;
    a.M = pl->Ml; a.N = pl->Nl; a.K = pl->Kl;
    a.tm = pl->tm; a.tn = pl->tn; a.t = pl->t; a.ipt = pl->ipt;
    a.sk_tiles = pl->sk_tiles; a.g_sk = pl->g_sk;
    a.sk_iters = pl->sk_tiles * pl->ipt;
    a.sk_q = pl->sk_q; a.sk_r = pl->sk_r;
    a.grid = pl->grid;
    a.sk_first = pl->sk_first ? 1 : 0;
    a.dp_only = pl->g_sk == 0 ? 1 : 0;
    a.alpha = alpha;
    a.beta = beta;
    a.out_dtype = pl->out;
    a.vec_a = 16;
    a.vec_b = 16;
    if (pl->ws_bytes) {
        unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
        a.err = reinterpret_cast<int32_t*>(ws);
        a.flags = reinterpret_cast<int32_t*>(ws + pl->flags_off);
        a.partials = reinterpret_cast<float*>(ws + pl->partials_off);
    }
    a.trace = trace;
    a.trace_per_wg = trace ? pl->max_segs : 0;
    a.spin_limit = 1 << 22;
    if (pl->grid == 0) return SKGEMM_OK;
    const int rc = launch_gemm(pl->dtype, pl->akc, pl->bkc, a, pl->grid, stream);
    return rc == int(hipSuccess) ? SKGEMM_OK : SKGEMM_ERR_HIP;
}

skgemm_status_t skgemm_run(skgemm_plan_t plan, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                           int64_t ldc, float alpha, float beta, const float* scale_a, const float* scale_b,
                           void* workspace, size_t ws_bytes, hipStream_t stream) {
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, nullptr, 0,
                    stream);
}

skgemm_status_t skgemm_run_traced(skgemm_plan_t plan, const void* A, int64_t lda, const void* B, int64_t ldb,
                                  void* C, int64_t ldc, float alpha, float beta, const float* scale_a,
                                  const float* scale_b, void* workspace, size_t ws_bytes, int32_t* trace,
                                  size_t trace_records, hipStream_t stream) {
    if (!trace) return SKGEMM_ERR_INVALID_ARG;
    return run_impl(plan, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes, trace,
                    trace_records, stream);
}

skgemm_status_t skgemm_plan_info(skgemm_plan_t pl, int64_t* info, int32_t n) {
    if (!pl || !info || n < 0) return SKGEMM_ERR_INVALID_ARG;
    const int64_t v[20] = {pl->Ml, pl->Nl, pl->Kl, pl->swapped ? 1 : 0, pl->BM, pl->BN, pl->BK, pl->tm, pl->tn,
                           pl->t, pl->ipt, pl->policy, pl->sk_tiles, pl->g_sk, pl->grid, pl->sk_first ? 1 : 0,
                           pl->p, pl->hybrid_min_waves, pl->akc ? 1 : 0, pl->bkc ? 1 : 0};
    for (int i = 0; i < n && i < 20; ++i) info[i] = v[i];
    return SKGEMM_OK;
}

skgemm_status_t skgemm_model_constants(skgemm_plan_t pl, double* abcd) {
    if (!pl || !abcd) return SKGEMM_ERR_INVALID_ARG;
    for (int i = 0; i < 4; ++i) abcd[i] = pl->model[i];
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
