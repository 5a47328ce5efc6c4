"""Benchmark: Stream-K vs data-parallel tiles on the BF16 shape sweep (one MI355X).

One step = one pass of the Stream-K GEMM (automatic policy: data-parallel
waves plus a Stream-K remainder) over the 1000-shape BF16 sweep: M, N, K
log-uniform in [128, 8192], half of them multiples of 128 and half with
+1..127 offsets, A and B iid N(0, 1) in bf16, FP32 accumulation, bf16 output.
Inputs for every shape are resident in HBM before timing starts (distinct
buffers per shape).  Plans are built once before the timed region.

Printed JSON line (rank 0):
  value        whole-sweep throughput of the Stream-K path, TFLOP/s
               (2*M*N*K useful flops over the wall time of the step)
  roofline     the dominant kernel (the BF16 Stream-K kernel) against the
               dense BF16 MFMA peak: achieved = flops per launch / average
               launch duration from HIP events around every launch
  dp_*         the same kernel with the data-parallel policy (one workgroup
               per tile) over the same shapes: the paper's baseline
  sk_over_dp_* per-shape speedups (geomean / min / median / max), over all
               shapes and over the quantisation-bound subset (tiles fill
               less than 90% of the last wave), warm (resident caches) and
               cold (L2 and MALL flushed before each launch)
  large_shapes BF16 4096^3 and 8192^3 with the automatic policy (TFLOP/s,
               % of the dense BF16 peak)
  cpu_baseline the FP64 oracle on the host cores over a bounded sample of
               the sweep
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TFLOP/s & % MFMA peak, Stream-K vs data-parallel tiles, bf16 shape sweep"

# HBM bytes per GEMM kernel launch of the sweep, from two rocprofv3 PMC runs (FETCH_SIZE, WRITE_SIZE,
# each scaled by its reading for a plain 256 MiB copy); valid only for the kernel sources
# they were taken on, identified by the hash below (see profiles/skgemm_bf16_sweep_hbm_traffic.md).
TRAFFIC_BYTES_PER_LAUNCH = 60.93e6
TRAFFIC_SOURCES_SHA256 = "5d9a6fb7e5a2408e"


def kernel_sources_hash() -> str:
    """Hash of the kernel sources' code (comments and blank lines left out, so
    that a comment edit does not invalidate counters taken on the same code)."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2212_08964_amd", "csrc", "*"))):
        if f.endswith((".hpp", ".hip", ".h", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f) as fh:
                text = fh.read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            code = [ln.split("//", 1)[0].rstrip() for ln in text.splitlines()]
            h.update("\n".join(ln for ln in code if ln.strip()).encode())
    return h.hexdigest()[:16]
PEAK_BF16_TFLOPS = 2516.6      # MI355X dense BF16 MFMA, 256 CU x 4096 flop/clk x 2.4 GHz
HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shapes", type=int, default=1000)
    ap.add_argument("--shape-seed", type=int, default=0,
                    help="seed of the sweep's shapes (the benchmark is seed 0; others check planner rules "
                         "on shapes they were not measured on)")
    ap.add_argument("--reps", type=int, default=8,
                    help="back-to-back launches per timed round for the per-shape ratios (best of 3 rounds)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-shape", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the BF16 4096^3 and 8192^3 timings")
    ap.add_argument("--no-waits", action="store_true", help="skip the timed pass that measures fix-up waits")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the passes")
    ap.add_argument("--profile-policy", default="auto", choices=["auto", "dp"],
                    help="with --profile-steps: which pass to run (the automatic policy or the DP baseline)")
    ap.add_argument("--profile-shape", default="",
                    help="MxNxK: run only this BF16 GEMM (automatic policy) --profile-steps times, for profilers")
    ap.add_argument("--relayout", default="auto", choices=["auto", "never"],
                    help="operand re-layout of misaligned rows: the planner's rule, or never")
    ap.add_argument("--dump", default="", help="write per-shape timings (JSON lines) to this path")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many Stream-K steps (for profiler runs) and print timings")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the sweep: time the other workloads (FP32 plain GEMM, precision ladder, "
                         "grouped launch under a graph, autograd forward+backward), one JSON line each")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="with --profile-steps: then one plain device copy of this many MiB, the reference "
                         "that scales the HBM byte counters")
    return ap.parse_args()


class Case:
    __slots__ = ("M", "N", "K", "A", "B", "C", "sk", "dp", "flops", "bytes", "fixup_bytes", "t", "p")


def build_cases(shapes, torch, sk, relayout=0):
    cases = []
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    for (M, N, K) in shapes:
        c = Case()
        c.M, c.N, c.K = M, N, K
        c.A = torch.randn((M, K), generator=gen, device=dev, dtype=torch.float32).to(torch.bfloat16)
        c.B = torch.randn((K, N), generator=gen, device=dev, dtype=torch.float32).to(torch.bfloat16)
        c.C = torch.empty((M, N), device=dev, dtype=torch.bfloat16)
        c.sk = sk.Plan(M, N, K, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.BF16, sk.BF16, policy="auto",
                       relayout=relayout)
        info = c.sk.info()
        # the baseline: the same kernel and tile with one workgroup per tile
        c.dp = sk.Plan(M, N, K, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.BF16, sk.BF16, policy="dp",
                       tile=info["tile"], relayout=relayout)
        c.t, c.p = info["t"], info["p"]
        c.flops = 2.0 * M * N * K
        c.bytes = 2 * (M * K + K * N + M * N)       # read A and B once, write C once (bf16)
        # the method's own traffic: every partial segment writes one FP32 tile
        # and its reducer reads it back
        n_partials = sum(1 for r in c.sk.schedule() if r[5] == 1)
        c.fixup_bytes = 2 * n_partials * info["BM"] * info["BN"] * 4
        cases.append(c)
    return cases


def make_launcher(c, plan, ws, stream):
    """Pre-resolved C-ABI call for one GEMM (argument marshalling only)."""
    import ctypes
    from paper_2212_08964_amd import skgemm as sk
    L = sk.lib()
    nws = plan.workspace_size()
    args = (plan.handle, ctypes.c_void_p(c.A.data_ptr()), c.K, ctypes.c_void_p(c.B.data_ptr()), c.N,
            ctypes.c_void_p(c.C.data_ptr()), c.N, ctypes.c_float(1.0), ctypes.c_float(0.0), None, None,
            ctypes.c_void_p(ws.data_ptr()) if nws else None, nws, ctypes.c_void_p(stream))
    fn = L.skgemm_run

    def launch():
        st = fn(*args)
        if st != 0:
            raise sk.SkgemmError(st, "skgemm_run")
    return launch


def fixup_waits(cases, ws, stream, torch, np):
    """Time spent in the fix-up waits over the sweep's Stream-K plans, from
    one timed run each (segment stamps of the device's real-time clock): the
    share of the Stream-K workgroups' time spent waiting for peers' partial
    tiles, split by how many workgroups share a tile (the paper expects the
    waits to be negligible when at most two do, and not when three or more
    finish their shares of one tile together)."""
    from paper_2212_08964_amd import skgemm as sk
    hz = sk.realtime_hz()
    agg = {"le2": [0.0, 0.0, 0], "ge3": [0.0, 0.0, 0]}
    waits_us = []
    for c in cases:
        info = c.sk.info()
        if not info["g_sk"]:
            continue
        cap = c.sk.trace_capacity()
        tr = torch.full((cap * 8,), -1, dtype=torch.int32, device="cuda:0")
        tm = torch.zeros((cap * 7,), dtype=torch.int64, device="cuda:0")
        args = (c.A.data_ptr(), c.K, c.B.data_ptr(), c.N, c.C.data_ptr(), c.N, 1.0, 0.0, None, None,
                ws.data_ptr(), c.sk.workspace_size())
        c.sk.run(*args, stream=stream)
        c.sk.run_timed(*args, tr.data_ptr(), tm.data_ptr(), cap, stream=stream)
        torch.cuda.synchronize()
        recs = tr.cpu().numpy().reshape(-1, 8)
        st = tm.cpu().numpy().reshape(-1, 7)[:, :5].astype(np.float64) / hz * 1e6
        used = recs[:, 0] >= 0
        recs, st = recs[used], st[used]
        contrib = {}
        for r in recs:
            if r[0] < info["g_sk"] and r[2] < info["sk_tiles"]:
                contrib.setdefault(int(r[2]), set()).add(int(r[0]))
        key = "le2" if max((len(v) for v in contrib.values()), default=1) <= 2 else "ge3"
        busy = wait = 0.0
        for wg in range(info["g_sk"]):
            m = recs[:, 0] == wg
            if not m.any():
                continue
            busy += st[m, 4].max() - st[m, 0].min()
            w = float((st[m, 3] - st[m, 2]).sum())
            wait += w
            if w > 0:
                waits_us.append(w)
        agg[key][0] += wait
        agg[key][1] += busy
        agg[key][2] += 1
    out = {"plans": sum(v[2] for v in agg.values()),
           "clock_hz": hz,
           "note": "wait = stamps between the partial stores and the end of the fix-up waits, summed over the "
                   "Stream-K workgroups; share = wait / (their first-segment start to last-segment end)"}
    for k, (w, b, n) in agg.items():
        out[f"share_{k}_contributors"] = round(w / b, 4) if b else None
        out[f"plans_{k}_contributors"] = n
    if waits_us:
        out["median_wait_us_of_waiting_workgroups"] = round(float(np.median(waits_us)), 3)
    return out


def cpu_baseline(shapes, budget_s):
    """FP64 oracle on the host over a prefix of the sweep (bounded by budget_s)."""
    import numpy as np
    from oracle import gemm as og
    g = np.random.default_rng(1)
    # smallest-first prefix of a fixed random order of the sweep, so the sample
    # spans many shapes within the budget
    order = g.permutation(len(shapes))
    flops, secs, used = 0.0, 0.0, []
    threads = og.num_threads()
    for i in order:
        M, N, K = shapes[i]
        est = 2.0 * M * N * K
        if used and secs + est / max(flops / max(secs, 1e-9), 1e9) > budget_s:
            continue
        A = g.standard_normal((M, K))
        B = g.standard_normal((K, N))
        t0 = time.perf_counter()
        og.gemm_f64(A, B)
        secs += time.perf_counter() - t0
        flops += est
        used.append(int(i))
        if secs >= budget_s or len(used) >= 64:
            break
    return {"value": flops / secs / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(used)} shapes of the sweep (random order, fitted to a {budget_s:.0f} s budget), "
                      f"{flops / 1e9:.1f} GFLOP in {secs:.1f} s, FP64 triple loop with OpenMP over rows"}


PEAKS = {"f32": 157.3, "bf16": PEAK_BF16_TFLOPS, "f16": PEAK_BF16_TFLOPS, "fp8": 5033.2, "f64": 78.6}


def _best_us(fn, reps, rounds=3):
    """Best-of-rounds mean launch time (us) of `reps` back-to-back calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(rounds):
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e3 / reps)
    return best


def _best_us_alternating(fns, reps, rounds=3):
    """_best_us of several launch functions, their timed rounds interleaved so
    that no function always runs first (clock ramps and cache state)."""
    import torch
    for f in fns:
        f()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = [float("inf")] * len(fns)
    for _ in range(rounds):
        for i, f in enumerate(fns):
            e0.record()
            for _ in range(reps):
                f()
            e1.record()
            e1.synchronize()
            best[i] = min(best[i], e0.elapsed_time(e1) * 1e3 / reps)
    return best


def suite(args):
    """The non-sweep workloads, timed on one GPU (inputs resident, plans built beforehand)."""
    import torch
    import workloads as W
    from paper_2212_08964_amd import skgemm as sk
    from paper_2212_08964_amd import autotune
    from paper_2212_08964_amd.autograd import skgemm_matmul
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)

    def emit(d):
        print(json.dumps(d), flush=True)

    def reps_for(flops):
        return int(min(200, max(5, 2e12 / max(flops, 1.0))))

    # FP32 plain GEMM, 384 x 384 x 1024 (nine 128 x 128 tiles)
    a, b = W.plain_f32(seed=0)
    A = torch.from_numpy(a).to(dev)
    B = torch.from_numpy(b).to(dev)
    C = torch.empty((384, 384), device=dev)
    fl = 2.0 * 384 * 384 * 1024
    row = {"workload": "fp32 384x384x1024", "dtype": "f32"}
    for pol in ("auto", "dp"):
        us = _best_us(lambda: sk.matmul(A, B, out=C, policy=pol), 200)
        row[pol + "_us"] = round(us, 2)
        row[pol + "_tflops"] = round(fl / us / 1e6, 3)
    info = sk.get_plan(384, 384, 1024, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.F32, sk.F32).info()
    row["auto_plan"] = {k: info[k] for k in ("policy_name", "g_sk", "BM", "BN", "BK")}
    emit(row)

    # precision ladder: bf16, fp16 and fp8 (per-tensor scales) at M=N=K in {1024, 4096, 8192}
    # and the skinny 128 x 8192 x 8192
    for (M, N, K) in [(1024, 1024, 1024), (4096, 4096, 4096), (8192, 8192, 8192), (128, 8192, 8192)]:
        A32 = torch.randn((M, K), generator=gen, device=dev)
        B32 = torch.randn((K, N), generator=gen, device=dev)
        fl = 2.0 * M * N * K
        for name in ("bf16", "f16", "fp8"):
            if name == "fp8":
                qa, sa = sk.quantize_e4m3(A32, "row")
                qb, sb = sk.quantize_e4m3(B32, "col")
                C = torch.empty((M, N), device=dev, dtype=torch.float32)
                ops = {pol: (lambda pol=pol: sk.matmul(qa, qb, out=C, scale_a=sa, scale_b=sb, policy=pol))
                       for pol in ("auto", "dp")}
                in_bytes, out_bytes = M * K + K * N, 4 * M * N
            else:
                dt = torch.bfloat16 if name == "bf16" else torch.float16
                Ai, Bi = A32.to(dt), B32.to(dt)
                C = torch.empty((M, N), device=dev, dtype=dt)
                ops = {pol: (lambda pol=pol: sk.matmul(Ai, Bi, out=C, policy=pol)) for pol in ("auto", "dp")}
                in_bytes, out_bytes = 2 * (M * K + K * N), 2 * M * N
            row = {"workload": f"{name} {M}x{N}x{K}", "dtype": name}
            times = _best_us_alternating([ops["auto"], ops["dp"]], reps_for(fl))
            for (pol, fn), us in zip(ops.items(), times):
                tf = fl / us / 1e6
                row[pol + "_us"] = round(us, 2)
                row[pol + "_tflops"] = round(tf, 1)
                row[pol + "_pct_peak"] = round(100 * tf / PEAKS[name], 2)
                row[pol + "_hbm_gbs"] = round((in_bytes + out_bytes) / us / 1e3, 1)
            if name == "fp8":
                us_q = _best_us(lambda: (sk.quantize_e4m3(A32, "row", out=qa, scale=sa),
                                         sk.quantize_e4m3(B32, "col", out=qb, scale=sb)), 20)
                qbytes = 4 * (M * K + K * N) * 2 + (M * K + K * N)   # two FP32 passes (absmax, cast) + fp8 out
                row["quantize_us"] = round(us_q, 2)
                row["quantize_hbm_gbs"] = round(qbytes / us_q / 1e3, 1)
            if name == "bf16":
                # context: the vendor library GEMM (hipBLASLt through torch) on the same operands
                us_t = _best_us(lambda: torch.matmul(Ai, Bi, out=C), reps_for(fl))
                row["torch_matmul_us"] = round(us_t, 2)
                row["torch_matmul_tflops"] = round(fl / us_t / 1e6, 1)
            emit(row)
            del C
        del A32, B32
        torch.cuda.empty_cache()

    # FP64 (64 x 64 x 16 tiles, FP64 MFMA, FP64 fix-up) on the same shapes
    for (M, N, K) in [(1024, 1024, 1024), (4096, 4096, 4096), (8192, 8192, 8192), (128, 8192, 8192)]:
        A64 = torch.randn((M, K), generator=gen, device=dev, dtype=torch.float64)
        B64 = torch.randn((K, N), generator=gen, device=dev, dtype=torch.float64)
        C = torch.empty((M, N), device=dev, dtype=torch.float64)
        fl = 2.0 * M * N * K
        row = {"workload": f"f64 {M}x{N}x{K}", "dtype": "f64"}
        times = _best_us_alternating([lambda: sk.matmul(A64, B64, out=C, policy="auto"),
                                      lambda: sk.matmul(A64, B64, out=C, policy="dp")],
                                     int(min(50, max(3, 2e11 / fl))))
        for pol, us in zip(("auto", "dp"), times):
            tf = fl / us / 1e6
            row[pol + "_us"] = round(us, 2)
            row[pol + "_tflops"] = round(tf, 2)
            row[pol + "_pct_peak"] = round(100 * tf / PEAKS["f64"], 2)
        us_t = _best_us(lambda: torch.matmul(A64, B64, out=C), int(min(50, max(3, 2e11 / fl))))
        row["torch_matmul_us"] = round(us_t, 2)
        row["torch_matmul_tflops"] = round(fl / us_t / 1e6, 2)
        emit(row)
        del A64, B64, C
        torch.cuda.empty_cache()

    # grouped: 64 problems, N=4096, K=2048, M ~ Zipf(1.2) on [16, 4096], one launch under a graph
    Ms = W.zipf_ms(64, seed=0)
    N, K = 4096, 2048
    As = [torch.randn((m, K), generator=gen, device=dev).to(torch.bfloat16) for m in Ms]
    Bs = [torch.randn((K, N), generator=gen, device=dev).to(torch.bfloat16) for _ in Ms]
    Cs = [torch.empty((m, N), device=dev, dtype=torch.bfloat16) for m in Ms]
    fl = sum(2.0 * m * N * K for m in Ms)
    best, tried = autotune.tune_grouped(As, Bs, Cs, reps=10)
    _, table = sk.grouped_matmul(As, Bs, Cs, **best)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        sk.grouped_matmul(As, Bs, Cs, table=table, **best)
    torch.cuda.synchronize()
    us_graph = _best_us(graph.replay, 20)
    _, tdp = sk.grouped_matmul(As, Bs, Cs, policy="dp")
    us_gdp = _best_us(lambda: sk.grouped_matmul(As, Bs, Cs, table=tdp, policy="dp"), 20)
    us_seq = _best_us(lambda: [sk.matmul(a_, b_, out=c_, policy="dp") for a_, b_, c_ in zip(As, Bs, Cs)], 5)
    emit({"workload": "grouped bf16: 64 problems N=4096 K=2048 M~Zipf(1.2) on [16,4096]", "dtype": "bf16",
          "gflop": round(fl / 1e9, 1), "autotuned": best,
          "candidates_us": {k: round(v, 1) for k, v in tried.items()},
          "graph_replay_us": round(us_graph, 1), "graph_replay_tflops": round(fl / us_graph / 1e6, 1),
          "grouped_dp_us": round(us_gdp, 1), "grouped_dp_tflops": round(fl / us_gdp / 1e6, 1),
          "sequential_dp_us": round(us_seq, 1), "sequential_dp_tflops": round(fl / us_seq / 1e6, 1)})
    del As, Bs, Cs
    torch.cuda.empty_cache()

    # autograd forward + backward (dA = dC B^T, dB = A^T dC) in bf16
    for (M, N, K) in [(2048, 2048, 8192), (256, 4096, 4096)]:
        A = torch.randn((M, K), generator=gen, device=dev).to(torch.bfloat16).requires_grad_()
        B = torch.randn((K, N), generator=gen, device=dev).to(torch.bfloat16).requires_grad_()
        dC = torch.randn((M, N), generator=gen, device=dev).to(torch.bfloat16)
        fl = 3 * 2.0 * M * N * K

        def step():
            A.grad = B.grad = None
            skgemm_matmul(A, B).backward(dC)
        us = _best_us(step, 20)
        # the same three products called directly (no autograd bookkeeping on the host):
        # the GPU's share of the step when the host-side graph work is the bound
        Cf = torch.empty((M, N), device=dev, dtype=torch.bfloat16)
        dA = torch.empty((M, K), device=dev, dtype=torch.bfloat16)
        dB = torch.empty((K, N), device=dev, dtype=torch.bfloat16)
        Ad, Bd = A.detach(), B.detach()
        us_k = _best_us(lambda: (sk.matmul(Ad, Bd, out=Cf), sk.matmul(dC, Bd.t(), out=dA),
                                 sk.matmul(Ad.t(), dC, out=dB)), 20)
        # the same step captured once in a HIP graph and replayed (no host work per product)
        from paper_2212_08964_amd.autograd import GraphedStep
        gstep = GraphedStep(Ad, Bd, dC)
        us_g = _best_us(gstep.replay, 20)
        emit({"workload": f"autograd bf16 {M}x{N}x{K} forward+backward", "dtype": "bf16",
              "ms": round(us / 1e3, 4), "tflops": round(fl / us / 1e6, 1),
              "pct_peak": round(100 * fl / us / 1e6 / PEAK_BF16_TFLOPS, 2),
              "three_gemms_ms": round(us_k / 1e3, 4), "three_gemms_tflops": round(fl / us_k / 1e6, 1),
              "graphed_step_ms": round(us_g / 1e3, 4), "graphed_step_tflops": round(fl / us_g / 1e6, 1)})
        del gstep


    # implicit-GEMM convolution: the 3x3 convolutions of ResNet-50's four stages and one 1x1
    # projection, batch 32, channels-last bf16; torch's convolution (MIOpen) on the same
    # channels-last tensors for context
    for (n, h, c, k, r, std) in [(32, 56, 64, 64, 3, 1), (32, 28, 128, 128, 3, 1), (32, 14, 256, 256, 3, 1),
                                 (32, 7, 512, 512, 3, 1), (32, 14, 1024, 256, 1, 1)]:
        pad = r // 2
        x = torch.randn((n, h, h, c), generator=gen, device=dev).to(torch.bfloat16)
        f = (torch.randn((k, r, r, c), generator=gen, device=dev) / (r * r * c) ** 0.5).to(torch.bfloat16)
        P = (h + 2 * pad - r) // std + 1
        y = torch.empty((n, P, P, k), device=dev, dtype=torch.bfloat16)
        fl = 2.0 * n * P * P * k * r * r * c
        ops = [lambda pol=pol: sk.conv2d(x, f, y, padding=(pad, pad), stride=(std, std), policy=pol)
               for pol in ("auto", "dp")]
        times = _best_us_alternating(ops, reps_for(fl))
        plan = sk.ConvPlan(n, h, h, c, k, r, r, (pad, pad), (std, std), ta=sk.BF16).info()
        row = {"workload": f"conv bf16 n{n} {h}x{h} c{c} k{k} {r}x{r} s{std}", "dtype": "bf16",
               "gemm_view": [plan["M"], plan["N"], plan["K"]],
               "auto_plan": {k_: plan[k_] for k_ in ("policy_name", "g_sk", "BM", "BN", "BK", "t")}}
        for pol, us in zip(("auto", "dp"), times):
            row[pol + "_us"] = round(us, 2)
            row[pol + "_tflops"] = round(fl / us / 1e6, 1)
        xt = x.permute(0, 3, 1, 2)              # NCHW view, channels-last memory
        ft = f.permute(0, 3, 1, 2)
        try:
            us_t = _best_us(lambda: torch.nn.functional.conv2d(xt, ft, padding=pad, stride=std), reps_for(fl))
            row["torch_conv2d_us"] = round(us_t, 2)
            row["torch_conv2d_tflops"] = round(fl / us_t / 1e6, 1)
        except RuntimeError as e:           # a convolution library without this case
            row["torch_conv2d_error"] = str(e)[:120]
        emit(row)


def profile_shape(args):
    """One BF16 GEMM (A, B, C row-major, N(0,1) inputs, automatic policy) run
    --profile-steps times back to back, for rocprofv3 kernel traces and
    counters of a single shape."""
    import torch
    from paper_2212_08964_amd import skgemm as sk
    M, N, K = (int(x) for x in args.profile_shape.lower().split("x"))
    c = Case()
    c.M, c.N, c.K = M, N, K
    c.A = torch.randn((M, K), device="cuda:0", dtype=torch.float32).to(torch.bfloat16)
    c.B = torch.randn((K, N), device="cuda:0", dtype=torch.float32).to(torch.bfloat16)
    c.C = torch.empty((M, N), device="cuda:0", dtype=torch.bfloat16)
    plan = sk.Plan(M, N, K, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.BF16, sk.BF16, policy="auto")
    ws = torch.zeros(max(plan.workspace_size(), 256), dtype=torch.uint8, device="cuda:0")
    f = make_launcher(c, plan, ws, torch.cuda.current_stream().cuda_stream)
    steps = max(1, args.profile_steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        f()
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    info = plan.info()
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy probe: {nb} bytes read, {nb} bytes written", flush=True)
    print(json.dumps({"shape": [M, N, K], "plan": {k: info[k] for k in ("policy_name", "tile", "g_sk", "grid", "stages")},
                      "launches": steps, "us_per_launch": round(us, 2),
                      "tflops": round(2.0 * M * N * K / (us * 1e-6) / 1e12, 1),
                      "algorithmic_bytes": 2 * (M * K + K * N + M * N)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (single-GPU build); --gpus must be 1"}))
        sys.exit(2)
    if args.suite:
        suite(args)
        return
    if args.profile_shape:
        profile_shape(args)
        return
    import numpy as np
    import torch
    import workloads as W
    from paper_2212_08964_amd import skgemm as sk

    shapes = W.sweep_shapes(args.shapes, seed=args.shape_seed)
    t0 = time.perf_counter()
    cases = build_cases(shapes, torch, sk, relayout=0 if args.relayout == "auto" else -1)
    plan_s = time.perf_counter() - t0
    # planning cost alone (host, microseconds per plan)
    tp = time.perf_counter()
    for (M, N, K) in shapes[:200]:
        sk.Plan(M, N, K, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.BF16, sk.BF16)
    plan_us = (time.perf_counter() - tp) / min(200, len(shapes)) * 1e6

    ws_bytes = max(max(c.sk.workspace_size(), c.dp.workspace_size()) for c in cases)
    ws = torch.zeros(max(ws_bytes, 256), dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream
    sk_launch = [make_launcher(c, c.sk, ws, sptr) for c in cases]
    dp_launch = [make_launcher(c, c.dp, ws, sptr) for c in cases]
    total_flops = sum(c.flops for c in cases)
    torch.cuda.synchronize()

    def run_pass(launchers):
        for f in launchers:
            f()

    if args.profile_steps:
        passes = dp_launch if args.profile_policy == "dp" else sk_launch
        for s in range(args.profile_steps):
            t1 = time.perf_counter()
            run_pass(passes)
            torch.cuda.synchronize()
            print(f"profile step {s}: {(time.perf_counter() - t1) * 1e3:.2f} ms", flush=True)
        if args.copy_probe_mib:
            nb = args.copy_probe_mib << 20
            src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            print(f"copy probe: {nb} bytes read, {nb} bytes written", flush=True)
        fix = 0 if args.profile_policy == "dp" else sum(c.fixup_bytes for c in cases)
        print(f"{args.profile_policy} pass: algorithmic bytes per step: {sum(c.bytes for c in cases) + fix} "
              f"(fix-up {fix}); launches per step: {len(cases)}", flush=True)
        return

    for _ in range(args.warmup):
        run_pass(sk_launch)
        run_pass(dp_launch)
    torch.cuda.synchronize()

    # ---- timed region: K steps of the Stream-K pass, HIP events on the launch
    # stream at its two ends only (events between launches would add their own
    # dispatch gaps to every launch)
    n = len(cases)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(args.steps):
        run_pass(sk_launch)
    end.record(stream)
    torch.cuda.synchronize()
    wall_ms = start.elapsed_time(end)
    ms_per_step = wall_ms / args.steps
    avg_launch_us = ms_per_step * 1e3 / n
    value = total_flops / (ms_per_step * 1e-3) / 1e12
    # the step is nothing but back-to-back launches of the GEMM kernel, so the
    # kernel's mean flops per launch over its mean launch duration is the same figure
    achieved = (total_flops / n) / (avg_launch_us * 1e-6) / 1e12

    # ---- the data-parallel baseline pass, timed the same way
    start.record(stream)
    for s in range(args.steps):
        run_pass(dp_launch)
    end.record(stream)
    torch.cuda.synchronize()
    dp_ms_per_step = start.elapsed_time(end) / args.steps
    dp_value = total_flops / (dp_ms_per_step * 1e-3) / 1e12

    # ---- the same passes replayed from HIP graphs (one graph of n launches per
    # policy, captured on a side stream; the replays run the same kernels with
    # the same arguments, without per-launch host work)
    graph = None
    if not args.no_graph:
        cap = torch.cuda.Stream()
        gl_sk = [make_launcher(c, c.sk, ws, cap.cuda_stream) for c in cases]
        gl_dp = [make_launcher(c, c.dp, ws, cap.cuda_stream) for c in cases]
        cap.wait_stream(stream)
        graphs = {}
        for name, ls in (("sk", gl_sk), ("dp", gl_dp)):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                run_pass(ls)
            graphs[name] = g
        torch.cuda.synchronize()
        gms = {}
        for name in ("sk", "dp", "sk", "dp"):
            graphs[name].replay()
            torch.cuda.synchronize()
            start.record(stream)
            for _ in range(args.steps):
                graphs[name].replay()
            end.record(stream)
            torch.cuda.synchronize()
            t = start.elapsed_time(end) / args.steps
            gms[name] = min(gms.get(name, t), t)
        graph = {"ms_per_step": round(gms["sk"], 4), "value": round(total_flops / (gms["sk"] * 1e-3) / 1e12, 3),
                 "dp_ms_per_step": round(gms["dp"], 4),
                 "dp_value": round(total_flops / (gms["dp"] * 1e-3) / 1e12, 3),
                 "note": "one pass per policy captured in a HIP graph and replayed (best of two timed blocks of "
                         "K replays)"}
        del graphs

    # ---- per-shape times, both policies in alternating rounds (no policy
    # always runs first).  Warm: median over 5 rounds of back-to-back launches
    # on resident buffers.  Cold: median over 5 single launches, each after a
    # 512 MiB write that evicts the L2 caches and the MALL.
    ratios = None
    if not args.no_per_shape:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        flush = torch.empty(512 << 18, dtype=torch.float32, device="cuda:0")
        rounds = 5
        w_sk, w_dp = np.zeros((n, rounds)), np.zeros((n, rounds))
        c_sk, c_dp = np.zeros((n, rounds)), np.zeros((n, rounds))
        for i in range(n):
            for r in range(rounds):
                for arr, f in ((w_sk, sk_launch[i]), (w_dp, dp_launch[i])):
                    f()
                    e0.record(stream)
                    for _ in range(args.reps):
                        f()
                    e1.record(stream)
                    e1.synchronize()
                    arr[i, r] = e0.elapsed_time(e1) / args.reps
                for arr, f in ((c_sk, sk_launch[i]), (c_dp, dp_launch[i])):
                    flush.fill_(float(r))
                    e0.record(stream)
                    f()
                    e1.record(stream)
                    e1.synchronize()
                    arr[i, r] = e0.elapsed_time(e1)
        t_sk, t_dp = np.median(w_sk, axis=1), np.median(w_dp, axis=1)
        tc_sk, tc_dp = np.median(c_sk, axis=1), np.median(c_dp, axis=1)
        del flush
        ratios = t_dp / t_sk
        ratios_cold = tc_dp / tc_sk
        qb = np.array([c.t / (c.p * math.ceil(c.t / c.p)) < 0.9 for c in cases])
        if args.dump:
            with open(args.dump, "w") as fh:
                for c, a_, b_, ac, bc in zip(cases, t_sk, t_dp, tc_sk, tc_dp):
                    info = c.sk.info()
                    fh.write(json.dumps({"M": c.M, "N": c.N, "K": c.K, "t": c.t, "ipt": info["ipt"],
                                         "tile": info["BM"], "waves": info["waves"], "policy": info["policy_name"],
                                         "g": info["g_sk"], "sk_us": a_ * 1e3, "dp_us": b_ * 1e3,
                                         "sk_cold_us": ac * 1e3, "dp_cold_us": bc * 1e3,
                                         "gflop": c.flops / 1e9}) + "\n")

        def stats(r):
            return {"geomean": float(np.exp(np.mean(np.log(r)))), "min": float(r.min()),
                    "median": float(np.median(r)), "max": float(r.max()), "n": int(r.size)}
        flops_arr = np.array([c.flops for c in cases])
        per_shape = {
            "timing": f"warm: median of {rounds} rounds of {args.reps} back-to-back launches; cold: median of "
                      f"{rounds} single launches each after a 512 MiB write (L2 and MALL evicted)",
            "all": stats(ratios),
            "quantization_bound": stats(ratios[qb]) if qb.any() else None,
            "cold_all": stats(ratios_cold),
            "cold_quantization_bound": stats(ratios_cold[qb]) if qb.any() else None,
            "sk_tflops_geomean": float(np.exp(np.mean(np.log(flops_arr / (t_sk * 1e-3) / 1e12)))),
            "dp_tflops_geomean": float(np.exp(np.mean(np.log(flops_arr / (t_dp * 1e-3) / 1e12)))),
            "sk_tflops_max": float((flops_arr / (t_sk * 1e-3) / 1e12).max()),
        }
    torch.cuda.synchronize()

    waits = None if args.no_waits else fixup_waits(cases, ws, sptr, torch, np)

    # ---- the large-shape target: BF16 4096^3 and 8192^3 (automatic policy)
    large = {}
    if not args.no_large:
        for L_ in (4096, 8192):
            lc = Case()
            lc.M = lc.N = lc.K = L_
            lc.A = torch.randn((L_, L_), device="cuda:0", dtype=torch.float32).to(torch.bfloat16)
            lc.B = torch.randn((L_, L_), device="cuda:0", dtype=torch.float32).to(torch.bfloat16)
            lc.C = torch.empty((L_, L_), device="cuda:0", dtype=torch.bfloat16)
            plan = sk.Plan(L_, L_, L_, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.ROW_MAJOR, sk.BF16, sk.BF16, policy="auto")
            lws = torch.zeros(max(plan.workspace_size(), 256), dtype=torch.uint8, device="cuda:0")
            f = make_launcher(lc, plan, lws, sptr)
            for _ in range(3):
                f()
            reps = 20 if L_ == 4096 else 8
            times = []
            for _ in range(5):
                start.record(stream)
                for _ in range(reps):
                    f()
                end.record(stream)
                end.synchronize()
                times.append(start.elapsed_time(end) / reps)
            ms = float(np.median(times))
            tf = 2.0 * L_ ** 3 / (ms * 1e-3) / 1e12
            info = plan.info()
            # the shader clock under this load, from one timed run of the same plan
            # (shader-clock ticks over real time, summed over its segments)
            cap = plan.trace_capacity()
            tr = torch.full((cap * 8,), -1, dtype=torch.int32, device="cuda:0")
            tm = torch.zeros((cap * 7,), dtype=torch.int64, device="cuda:0")
            plan.run_timed(lc.A.data_ptr(), L_, lc.B.data_ptr(), L_, lc.C.data_ptr(), L_, 1.0, 0.0, None, None,
                           lws.data_ptr(), lws.numel(), tr.data_ptr(), tm.data_ptr(), cap, stream=sptr)
            torch.cuda.synchronize()
            st = tm.cpu().numpy().reshape(-1, 7)[tr.cpu().numpy().reshape(-1, 8)[:, 0] >= 0].astype(np.float64)
            ghz = float((st[:, 6] - st[:, 5]).sum() / ((st[:, 4] - st[:, 0]).sum() / sk.realtime_hz()) / 1e9)
            large[f"bf16_{L_}"] = {"tflops": round(tf, 1), "pct_peak": round(100.0 * tf / PEAK_BF16_TFLOPS, 2),
                                   "us": round(ms * 1e3, 2), "policy": info["policy_name"],
                                   "tile": list(info["tile"]), "shader_ghz": round(ghz, 3),
                                   "pct_peak_at_shader_clock": round(100.0 * tf / (PEAK_BF16_TFLOPS * ghz / 2.4), 2)}
            del lc, lws
        torch.cuda.synchronize()

    sk_bytes = [c.bytes + c.fixup_bytes for c in cases]
    # per-shape roofline: each GEMM at max(flops / MFMA peak, algorithmic bytes / HBM bandwidth)
    roof_ms = sum(max(c.flops / (PEAK_BF16_TFLOPS * 1e12), b / (HBM_GBS * 1e9)) for c, b in zip(cases, sk_bytes))
    roof_ms *= 1e3

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "bf16 shape sweep: 1000 GEMMs, M,N,K log-uniform in [128,8192] "
                               "(half multiples of 128, half +1..127), A,B iid N(0,1) bf16, FP32 accumulate, "
                               "bf16 out, row-major",
                   "n_shapes": n, "shape_seed": args.shape_seed, "policy": "auto (DP waves + Stream-K remainder)",
                   "baseline": "same kernel and tile, policy=dp (one workgroup per tile)",
                   "tiles": "256x256x64, or 128x128x64 (4 or 8 waves) where the planner predicts it faster "
                            "(same tile for both)",
                   "relayout": {"auto": "planner's rule (misaligned operand rows copied to 128-byte lines "
                                        "when predicted faster; the copy is timed)",
                                "never": "off"}[args.relayout],
                   "total_gflop": round(total_flops / 1e9, 1), "parallelism": "single GPU"},
        "pct_mfma_peak": round(100.0 * value / PEAK_BF16_TFLOPS, 2),
        "dp_value": round(dp_value, 3),
        "dp_ms_per_step": round(dp_ms_per_step, 4),
        "sk_over_dp_aggregate": round(value / dp_value, 4),
        "sk_over_dp_per_shape": ratios is not None and per_shape or None,
        "graph_replay": graph,
        "large_shapes": large or None,
        "fixup_waits": waits,
        "plan_us_per_gemm": round(plan_us, 2),
        "setup_s": round(plan_s, 2),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4),
                     "traffic": TRAFFIC_BYTES_PER_LAUNCH if kernel_sources_hash() == TRAFFIC_SOURCES_SHA256 else None,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": round(sum(sk_bytes) / n),
                     "algorithmic_bytes_note": "A and B read once, C written once (bf16), plus the fix-up: "
                                               "2 x partial segments x BM x BN x 4 bytes",
                     "fixup_bytes_per_launch": round(sum(c.fixup_bytes for c in cases) / n),
                     "per_shape_roofline_ms": round(roof_ms, 4),
                     "per_shape_roofline_frac": round(roof_ms / ms_per_step, 4),
                     "kernel": "skgemm_kernel<BF16, A K-contiguous, B N-contiguous>",
                     "avg_launch_us": round(avg_launch_us, 3),
                     "flops_per_launch": round(total_flops / n, 1)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(shapes, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
