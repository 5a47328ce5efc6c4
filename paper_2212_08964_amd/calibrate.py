"""Measure the grid-size model constants on the local GPU.

The Analytical Modeling subsection models the runtime of one tile-producing
workgroup as a + b*[peers > 1] + c*iters_per_cta + d*(peers - 1), with the
constants found by microbenchmarks once per blocking factor, data type and
GPU.  This script runs basic Stream-K with forced grid sizes over synthetic
problems (tile counts t, iterations per tile ipt, grid sizes g = s*t that
split each tile into s equal parts), times back-to-back launches with HIP
events, and fits (a, b, c, d) by least squares.  It
prints the constants normalised to c = 1, in the form the library's model
table uses.

A second mode fits all five constants of every 16-bit GEMM tile at once on a
seeded sweep of random shapes (log-uniform M, N, K in [128, 8192], half of
them multiples of 128, half with +1..127 offsets): each shape is planned with
the automatic policy on each tile, timed, and (a, b, c, d, e) are fitted by
least squares on relative error to the planner's estimate of those plans,
which is linear in the constants once a plan is resolved.  The microbenchmark
grids above pin the constants of one workgroup per CU on tile-aligned
problems; the sweep fit reports how well a set of constants predicts the
shapes the planner meets (ragged edges, co-resident workgroups, hybrids).
Constants fitted this way were measured in the library and not adopted:
fitted on warm, repeated timings, they chose splits that lost in a pass of
distinct, cold GEMMs.

Usage: python -m paper_2212_08964_amd.calibrate [bf16|f16|f32|f64] [BMxBNxBK[xWAVES], e.g. 128x128x64x8]
       python -m paper_2212_08964_amd.calibrate sweep [n_shapes] [seed]
"""
from __future__ import annotations

import math
import sys


def model_terms(t, ipt, g):
    ipc = math.ceil(t * ipt / g)
    peers = math.ceil(ipt / ipc)
    return [1.0, 1.0 if peers > 1 else 0.0, float(ipc), float(peers - 1)]


def estimate_terms(info):
    """Coefficients of (a, b, c, d, e) in the planner's compute-time estimate
    of a resolved single-GEMM plan: data-parallel plans run ceil(t/p) waves,
    a partial wave at the per-iteration time interpolated between c (one
    busy slot) and e (all p slots busy); Stream-K plans pay a workgroup's
    data-parallel tiles, a, the fix-up terms b and d, and their share of
    iterations at the time for g_sk busy slots.  The estimate is the dot
    product of these coefficients with the constants."""
    t, ipt, p = info["t"], info["ipt"], info["p"]
    g, skt, grid = info["g_sk"], info["sk_tiles"], info["grid"]
    if t == 0:
        return None
    if g == 0:
        full, rem = divmod(t, p)
        f = min(1.0, rem / p)
        part = 1.0 if rem else 0.0
        return [full + part, 0.0, part * ipt * (1.0 - f), 0.0, full * ipt + part * ipt * f]
    ipc = math.ceil(skt * ipt / g)
    peers = max(1, math.ceil(ipt / ipc))
    dp_per_wg = math.ceil((t - skt) / grid)
    f = min(1.0, g / p)
    return [1.0 + dp_per_wg, 1.0 if peers > 1 else 0.0, (1.0 - f) * ipc, float(peers - 1),
            dp_per_wg * ipt + f * ipc]


def sweep_shapes(n, seed):
    """Log-uniform shapes in [128, 8192]: the first half rounded to multiples
    of 128, the second half a multiple of 128 plus 1..127."""
    import numpy as np
    g = np.random.default_rng(seed)
    d = np.exp(g.uniform(math.log(128), math.log(8192), size=(n, 3)))
    out = []
    for i in range(n):
        if i < n // 2:
            v = np.maximum(np.rint(d[i] / 128.0), 1) * 128
        else:
            v = np.floor(d[i] / 128.0) * 128 + g.integers(1, 128, size=3)
        out.append(tuple(int(x) for x in v))
    return out


SWEEP_TILES = [(256, 256, 64, 8), (128, 128, 64, 4), (128, 128, 64, 8), (64, 256, 64, 4), (256, 64, 64, 4)]


def fit_sweep(n=1000, seed=1, dtype="bf16", verbose=True):
    """Times every shape of the seeded sweep on every 16-bit GEMM tile (the
    automatic policy on that tile; a column-major B where the tile has no
    kernel for a row-major one) and fits (a, b, c, d, e) per tile.  Returns
    {tile: (constants, rms relative error of the fit, of the current
    constants, number of shapes)}."""
    import ctypes
    import numpy as np
    import torch

    from . import skgemm as sk
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    cdt = {"bf16": sk.BF16, "f16": sk.F16}[dtype]
    L = sk.lib()
    stream = torch.cuda.current_stream()
    ws = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    rows = {tile: ([], [], []) for tile in SWEEP_TILES}
    for n_done, (M, N, K) in enumerate(sweep_shapes(n, seed)):
        A = torch.randn((M, K), generator=gen, device="cuda").to(tdt)
        Bk = torch.randn((K, N), generator=gen, device="cuda").to(tdt)
        Bn = None
        C = torch.empty((M, N), device="cuda", dtype=tdt)
        for tile in SWEEP_TILES:
            lb, B = sk.ROW_MAJOR, Bk
            try:
                plan = sk.Plan(M, N, K, ta=cdt, tc=cdt, policy="auto", tile=tile)
            except sk.SkgemmError:
                try:
                    plan = sk.Plan(M, N, K, lb=sk.COL_MAJOR, ta=cdt, tc=cdt, policy="auto", tile=tile)
                except sk.SkgemmError:
                    continue
                if Bn is None:
                    Bn = Bk.t().contiguous()
                lb, B = sk.COL_MAJOR, Bn
            info = plan.info()
            terms = estimate_terms(info)
            if terms is None:
                continue
            nws = plan.workspace_size()
            if nws > ws.numel():
                torch.cuda.synchronize()
                ws = torch.zeros(nws, dtype=torch.uint8, device="cuda")
            args = (plan.handle, ctypes.c_void_p(A.data_ptr()), K, ctypes.c_void_p(B.data_ptr()),
                    N if lb == sk.ROW_MAJOR else K, ctypes.c_void_p(C.data_ptr()), N, ctypes.c_float(1.0),
                    ctypes.c_float(0.0), None, None, ctypes.c_void_p(ws.data_ptr()), nws,
                    ctypes.c_void_p(stream.cuda_stream))
            st = L.skgemm_run(*args)
            if st:
                raise sk.SkgemmError(st, "skgemm_run")
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                e0.record()
                for _ in range(8):
                    L.skgemm_run(*args)
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e3 / 8)
            ts.sort()
            rows[tile][0].append(terms)
            rows[tile][1].append(ts[2])
            rows[tile][2].append(plan.model_constants())
        if verbose and n_done % 100 == 0:
            print(f"{n_done} shapes", flush=True)
        del A, Bk, Bn, C
    out = {}
    for tile, (X, y, cur) in rows.items():
        if not y:
            continue
        X, y, cur = np.array(X), np.array(y), np.array(cur)
        w = 1.0 / y
        coef = np.linalg.lstsq(X * w[:, None], y * w, rcond=None)[0]
        rms = lambda pred: float(np.sqrt(np.mean(np.log(y / np.maximum(pred, 1e-3)) ** 2)))
        out[tile] = (tuple(float(v) for v in coef), rms(X @ coef), rms(np.sum(X * cur, axis=1)), len(y))
    return out


def _launcher(sk, plan, A, B, C, ws, nws):
    """Pre-resolved C-ABI call on the current stream (argument marshalling done once), so
    that back-to-back launches are not limited by the host.  B is K x N row-major, or
    N x K row-major storage of a column-major K x N operand (plan.lb)."""
    import ctypes
    import torch
    L = sk.lib()
    args = (plan.handle, ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(B.data_ptr()), B.stride(0),
            ctypes.c_void_p(C.data_ptr()), C.stride(0), ctypes.c_float(1.0), ctypes.c_float(0.0), None, None,
            ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, nws,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    fn = L.skgemm_run

    def launch():
        st = fn(*args)
        if st:
            raise sk.SkgemmError(st, "skgemm_run")
    return launch


def measure(dtype="bf16", reps=20, verbose=True, tile=None):
    import numpy as np
    import torch

    from . import skgemm as sk
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16, "f32": torch.float32, "f64": torch.float64}[dtype]
    cdt = {"bf16": sk.BF16, "f16": sk.F16, "f32": sk.F32, "f64": sk.F64}[dtype]
    # a tile with no kernel for a row-major B (the tall one) is measured on a column-major B
    lb = sk.ROW_MAJOR
    try:
        probe = sk.Plan(256, 256, 64, ta=cdt, tc=cdt, policy="dp", tile=tile).info()
    except sk.SkgemmError:
        lb = sk.COL_MAJOR
        probe = sk.Plan(256, 256, 64, lb=lb, ta=cdt, tc=cdt, policy="dp", tile=tile).info()
    BM, BN, BK, p = probe["BM"], probe["BN"], probe["BK"], probe["p"]
    full_tile = probe["tile"]        # (BM, BN, BK, waves): pins this exact configuration
    rows, ys, grids = [], [], []
    for t in (1, 2, 4, 8, 16, 32, 64, 128, 192):
        for ipt in (4, 16, 64):
            tm = 1
            while tm * tm < t:
                tm *= 2
            tn = t // tm
            M, N, K = BM * tm, BN * tn, BK * ipt
            A = torch.randn(M, K, device="cuda").to(tdt)
            B = torch.randn((K, N) if lb == sk.ROW_MAJOR else (N, K), device="cuda").to(tdt)
            C = torch.empty(M, N, device="cuda", dtype=tdt)
            # grids that split every tile into s equal parts (s divides ipt): the
            # shares then start at the same k-offset in every tile, the form the
            # planner's automatic policy launches
            gs = [t * s for s in range(1, ipt + 1) if ipt % s == 0 and t * s <= p]
            for g in gs:
                plan = sk.Plan(M, N, K, lb=lb, ta=cdt, tc=cdt, policy="sk", force_g=g, tile=full_tile)
                nws = plan.workspace_size()
                ws = torch.zeros(max(nws, 256), dtype=torch.uint8, device="cuda")
                launch = _launcher(sk, plan, A, B, C, ws if nws else None, nws)
                launch()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                best = float("inf")
                for _ in range(3):
                    e0.record()
                    for _ in range(reps):
                        launch()
                    e1.record()
                    e1.synchronize()
                    best = min(best, e0.elapsed_time(e1) / reps * 1e3)
                rows.append(model_terms(t, ipt, g))
                ys.append(best)
                grids.append(g)
                if verbose:
                    print(f"t={t:4d} ipt={ipt:3d} g={g:4d}: {best:8.2f} us", flush=True)
    X = np.array(rows)
    y = np.array(ys)
    # a-d describe one workgroup per CU: fit them on grids no larger than the
    # CU count (the split rule switches to e beyond it)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    one = np.array([g <= cus for g in grids])
    coef, *_ = np.linalg.lstsq(X[one], y[one], rcond=None)
    a, b, c, d = (float(v) for v in coef)
    # e: per-iteration time with all p slots busy, from a data-parallel problem
    # of four full waves (four tiles per slot) at two depths.  A tile whose
    # plans of at most one workgroup per CU run a kernel of their own (the
    # three-stage small tile) is measured on one full wave of that kernel.
    big = sk.Plan(BM * 4 * p, BN, BK * 16, lb=lb, ta=cdt, tc=cdt, policy="dp", tile=full_tile).info()
    waves = 1 if big["stages"] != probe["stages"] else 4
    tw = []
    for ipt in (16, 64):
        t = waves * (cus if waves == 1 else p)
        tm = 1
        while tm * tm < t:
            tm *= 2
        tn = t // tm
        M, N, K = BM * tm, BN * tn, BK * ipt
        A = torch.randn(M, K, device="cuda").to(tdt)
        B = torch.randn((K, N) if lb == sk.ROW_MAJOR else (N, K), device="cuda").to(tdt)
        C = torch.empty(M, N, device="cuda", dtype=tdt)
        plan = sk.Plan(M, N, K, lb=lb, ta=cdt, tc=cdt, policy="dp", tile=full_tile)
        launch = _launcher(sk, plan, A, B, C, None, 0)
        launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            launch()
        e1.record()
        e1.synchronize()
        tw.append(e0.elapsed_time(e1) / 5 * 1e3 / waves)      # microseconds per wave
        if verbose:
            print(f"full waves: t={t} ipt={ipt}: {tw[-1]:.2f} us per wave", flush=True)
    e = (tw[1] - tw[0]) / (64 - 16)
    return (a / c, b / c, 1.0, d / c), (a, b, c, d, e), X[one], y[one]


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "sweep":
        n = int(sys.argv[2]) if len(sys.argv) > 2 else 1000
        seed = int(sys.argv[3]) if len(sys.argv) > 3 else 1
        for tile, (coef, rms_fit, rms_cur, cnt) in fit_sweep(n, seed).items():
            a, b, c, d, e = coef
            print(f"tile {tile}: a={a:.3f} b={b:.3f} c={c:.3f} d={d:.3f} e={e:.3f}  rms relative error "
                  f"{rms_fit:.3f} (current constants {rms_cur:.3f}) over {cnt} shapes", flush=True)
        return
    dtype = sys.argv[1] if len(sys.argv) > 1 else "bf16"
    tile = tuple(int(x) for x in sys.argv[2].split("x")) if len(sys.argv) > 2 else None
    norm, raw, X, y = measure(dtype, tile=tile)
    a, b, c, d, e = raw
    pred = X @ [a, b, c, d]
    import numpy as np
    err = float(np.sqrt(np.mean((pred - y) ** 2)))
    print(f"raw (us): a={a:.3f} b={b:.3f} c={c:.3f} d={d:.3f}  rms residual {err:.2f} us over {len(y)} runs")
    print(f"full occupancy (us per iteration): e={e:.3f}")
    print(f"normalised (c=1): a={norm[0]:.3f} b={norm[1]:.3f} c=1 d={norm[3]:.3f}")


if __name__ == "__main__":
    main()
