"""ctypes binding of libskgemm.so (the C ABI in include/skgemm.h).

Argument marshalling only: every step of the GEMM runs in the library's HIP
kernels.  The functions mirror the C entry points by name; ``matmul`` adds
the torch-tensor convenience layer (layouts from strides, the current HIP
stream, a cached zero-filled workspace per device and stream).

Loading fails loudly when the library has not been built: there is no other
execution path.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libskgemm.so")

# enums of include/skgemm.h
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_CAPACITY, ERR_HIP, ERR_TIMEOUT = range(7)
ROW_MAJOR, COL_MAJOR = 0, 1
F32, F16, BF16, F8E4M3, F64 = 0, 1, 2, 3, 4
POLICY = {"auto": 0, "dp": 1, "sk": 2, "dp_1tile_sk": 3, "2tile_sk_dp": 4, "paper": 5}
POLICY_NAME = {v: k for k, v in POLICY.items()}
ROLE_NAME = {0: "full", 1: "partial", 2: "owner"}

EXPORTED = [
    "skgemm_default_options", "skgemm_plan", "skgemm_workspace_size", "skgemm_run",
    "skgemm_trace_capacity", "skgemm_run_traced", "skgemm_plan_info", "skgemm_model_constants",
    "skgemm_schedule", "skgemm_check_device_error", "skgemm_plan_destroy", "skgemm_status_string",
    "skgemm_grouped_plan", "skgemm_grouped_table_size", "skgemm_grouped_table", "skgemm_grouped_run",
    "skgemm_grouped_run_traced", "skgemm_quantize_workspace_size", "skgemm_quantize_e4m3",
    "skgemm_run_timed", "skgemm_realtime_hz", "skgemm_run_noalloc",
    "skgemm_batched_plan", "skgemm_batched_run", "skgemm_batched_run_traced",
    "skgemm_conv_plan", "skgemm_conv_run", "skgemm_conv_run_traced",
]

INFO_FIELDS = ["M", "N", "K", "swapped", "BM", "BN", "BK", "tm", "tn", "t", "ipt", "policy",
               "sk_tiles", "g_sk", "grid", "sk_first", "p", "hybrid_min_waves", "a_kcontig", "b_kcontig", "G",
               "share", "coop_s", "occupancy", "waves", "batch", "pack_a", "pack_b", "fixup_ws_bytes",
               "stages"]
SHARE = {"proportional": 0, "leading": 1}
SHARE_NAME = {v: k for k, v in SHARE.items()}
FIXUP = {"auto": 0, "owner": 1}


class Options(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int), ("force_g", ctypes.c_int32), ("tile_m", ctypes.c_int32),
                ("tile_n", ctypes.c_int32), ("tile_k", ctypes.c_int32), ("hybrid_min_waves", ctypes.c_int32),
                ("num_cus", ctypes.c_int32), ("occupancy", ctypes.c_int32), ("raster_rows", ctypes.c_int32),
                ("xcds", ctypes.c_int32), ("share", ctypes.c_int32), ("fixup", ctypes.c_int32),
                ("tile_waves", ctypes.c_int32), ("spin_limit", ctypes.c_int32), ("relayout", ctypes.c_int32)]


class GroupArgs(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float)]


class ConvDesc(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("n", "h", "w", "c", "k", "r", "s", "pad_h", "pad_w", "stride_h",
                                               "stride_w", "dil_h", "dil_w")]


class SkgemmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2212_08964_amd/build.py")
                L = ctypes.CDLL(LIB_PATH)
                vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
                P = ctypes.POINTER
                L.skgemm_default_options.argtypes = [P(Options)]
                L.skgemm_default_options.restype = None
                L.skgemm_plan.argtypes = [P(vp), i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_int, P(Options)]
                L.skgemm_workspace_size.argtypes = [vp, P(sz)]
                L.skgemm_run.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.c_float, ctypes.c_float,
                                         vp, vp, vp, sz, vp]
                L.skgemm_trace_capacity.argtypes = [vp, P(sz)]
                L.skgemm_run_traced.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.c_float, ctypes.c_float,
                                                vp, vp, vp, sz, vp, sz, vp]
                L.skgemm_run_timed.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.c_float, ctypes.c_float,
                                               vp, vp, vp, sz, vp, vp, sz, vp]
                L.skgemm_realtime_hz.argtypes = [P(i64)]
                L.skgemm_batched_plan.argtypes = [P(vp), i64, i64, i64, i64, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(Options)]
                L.skgemm_batched_run.argtypes = [vp, vp, i64, i64, vp, i64, i64, vp, i64, i64, ctypes.c_float,
                                                 ctypes.c_float, vp, vp, vp, sz, vp]
                L.skgemm_batched_run_traced.argtypes = [vp, vp, i64, i64, vp, i64, i64, vp, i64, i64,
                                                        ctypes.c_float, ctypes.c_float, vp, vp, vp, sz, vp, sz, vp]
                L.skgemm_run_noalloc.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.c_float, ctypes.c_float,
                                                 vp, vp, vp]
                L.skgemm_conv_plan.argtypes = [P(vp), P(ConvDesc), ctypes.c_int, ctypes.c_int, P(Options)]
                L.skgemm_conv_run.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, sz, vp]
                L.skgemm_conv_run_traced.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, vp, sz, vp,
                                                     sz, vp]
                L.skgemm_plan_info.argtypes = [vp, P(i64), i32]
                L.skgemm_model_constants.argtypes = [vp, P(ctypes.c_double)]
                L.skgemm_schedule.argtypes = [vp, vp, sz, P(sz)]
                L.skgemm_check_device_error.argtypes = [vp, vp]
                L.skgemm_plan_destroy.argtypes = [vp]
                L.skgemm_status_string.argtypes = [ctypes.c_int]
                L.skgemm_status_string.restype = ctypes.c_char_p
                L.skgemm_grouped_plan.argtypes = [P(vp), i32, P(i64), P(i64), P(i64), ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(Options)]
                L.skgemm_grouped_table_size.argtypes = [vp, P(sz)]
                L.skgemm_grouped_table.argtypes = [vp, P(GroupArgs), vp, sz]
                L.skgemm_grouped_run.argtypes = [vp, vp, vp, sz, vp]
                L.skgemm_grouped_run_traced.argtypes = [vp, vp, vp, sz, vp, sz, vp]
                L.skgemm_quantize_workspace_size.argtypes = [P(sz)]
                L.skgemm_quantize_e4m3.argtypes = [vp, ctypes.c_int, i64, i64, ctypes.c_int, i64, vp, ctypes.c_int,
                                                   i64, vp, vp, sz, vp]
                for name in EXPORTED:
                    if name not in ("skgemm_default_options", "skgemm_status_string"):
                        getattr(L, name).restype = ctypes.c_int
                _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().skgemm_status_string(int(status)).decode()


def _check(status: int, what: str):
    if status != OK:
        raise SkgemmError(status, what)


def default_options() -> Options:
    o = Options()
    lib().skgemm_default_options(ctypes.byref(o))
    return o


class Plan:
    """Owns one skgemm_plan_t."""

    def __init__(self, M, N, K, la=ROW_MAJOR, lb=ROW_MAJOR, lc=ROW_MAJOR, ta=BF16, tc=None,
                 policy="auto", force_g=0, hybrid_min_waves=2, num_cus=0, occupancy=0, tile=None,
                 raster_rows=0, xcds=0, share="proportional", fixup="auto", spin_limit=0, relayout=0):
        self._h = ctypes.c_void_p()
        o = default_options()
        o.relayout = int(relayout)
        if tile:
            o.tile_m, o.tile_n, o.tile_k = (int(x) for x in tile[:3])
            if len(tile) > 3:
                o.tile_waves = int(tile[3])
        o.raster_rows, o.xcds = int(raster_rows), int(xcds)
        o.share = SHARE[share] if isinstance(share, str) else int(share)
        o.fixup = FIXUP[fixup] if isinstance(fixup, str) else int(fixup)
        o.policy = POLICY[policy] if isinstance(policy, str) else int(policy)
        o.force_g = int(force_g)
        o.hybrid_min_waves = int(hybrid_min_waves)
        o.num_cus = int(num_cus)
        o.spin_limit = int(spin_limit)
        o.occupancy = int(occupancy)
        tc = ta if tc is None else tc
        _check(lib().skgemm_plan(ctypes.byref(self._h), int(M), int(N), int(K), la, lb, lc, ta, ta, tc,
                                 ctypes.byref(o)), "skgemm_plan")
        self.M, self.N, self.K = int(M), int(N), int(K)
        self.la, self.lb, self.lc, self.ta, self.tc = la, lb, lc, ta, tc

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.skgemm_plan_destroy(h)
            self._h = ctypes.c_void_p()

    def workspace_size(self) -> int:
        # a plan is immutable: ask the library once
        ws = getattr(self, "_ws_bytes", None)
        if ws is None:
            n = ctypes.c_size_t()
            _check(lib().skgemm_workspace_size(self._h, ctypes.byref(n)), "skgemm_workspace_size")
            ws = self._ws_bytes = n.value
        return ws

    def trace_capacity(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().skgemm_trace_capacity(self._h, ctypes.byref(n)), "skgemm_trace_capacity")
        return n.value

    def info(self) -> dict:
        buf = (ctypes.c_int64 * len(INFO_FIELDS))()
        _check(lib().skgemm_plan_info(self._h, buf, len(INFO_FIELDS)), "skgemm_plan_info")
        d = dict(zip(INFO_FIELDS, list(buf)))
        d["policy_name"] = POLICY_NAME[d["policy"]]
        d["tile"] = (d["BM"], d["BN"], d["BK"], d["waves"])   # pins this exact configuration
        d["share_name"] = SHARE_NAME[d["share"]]
        return d

    def model_constants(self):
        """(a, b, c, d, e) of the plan's grid-size model, microseconds."""
        buf = (ctypes.c_double * 5)()
        _check(lib().skgemm_model_constants(self._h, buf), "skgemm_model_constants")
        return tuple(buf)

    def schedule(self):
        """Host-side schedule records: list of (wg, seq, tile, lo, hi, role, first_peer, last_peer)."""
        n = ctypes.c_size_t()
        _check(lib().skgemm_schedule(self._h, None, 0, ctypes.byref(n)), "skgemm_schedule")
        buf = (ctypes.c_int32 * (8 * max(1, n.value)))()
        _check(lib().skgemm_schedule(self._h, buf, n.value, ctypes.byref(n)), "skgemm_schedule")
        flat = list(buf)
        return [tuple(flat[8 * i:8 * i + 8]) for i in range(n.value)]

    def run(self, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0, scale_a=None, scale_b=None,
            workspace=None, ws_bytes=0, stream=None):
        """Raw pointers (ints) for every buffer; stream is a hipStream_t as int or None."""
        _check(lib().skgemm_run(self._h, A, int(lda), B, int(ldb), C, int(ldc), float(alpha), float(beta),
                                scale_a, scale_b, workspace, int(ws_bytes), stream), "skgemm_run")

    def run_traced(self, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes,
                   trace, trace_records, stream=None):
        _check(lib().skgemm_run_traced(self._h, A, int(lda), B, int(ldb), C, int(ldc), float(alpha),
                                       float(beta), scale_a, scale_b, workspace, int(ws_bytes), trace,
                                       int(trace_records), stream), "skgemm_run_traced")


    def run_noalloc(self, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0, scale_a=None, scale_b=None, stream=None):
        """skgemm_run on the library's own device array (no workspace argument)."""
        _check(lib().skgemm_run_noalloc(self._h, A, int(lda), B, int(ldb), C, int(ldc), float(alpha),
                                        float(beta), scale_a, scale_b, stream), "skgemm_run_noalloc")

    def run_timed(self, A, lda, B, ldb, C, ldc, alpha, beta, scale_a, scale_b, workspace, ws_bytes,
                  trace, times, trace_records, stream=None):
        _check(lib().skgemm_run_timed(self._h, A, int(lda), B, int(ldb), C, int(ldc), float(alpha),
                                      float(beta), scale_a, scale_b, workspace, int(ws_bytes), trace, times,
                                      int(trace_records), stream), "skgemm_run_timed")


def realtime_hz() -> int:
    """Ticks per second of the device clock the timed runs read."""
    v = ctypes.c_int64()
    _check(lib().skgemm_realtime_hz(ctypes.byref(v)), "skgemm_realtime_hz")
    return v.value


class BatchedPlan(Plan):
    """Owns one strided batched skgemm_plan_t (batch equal problems, one launch)."""

    def __init__(self, batch, M, N, K, la=ROW_MAJOR, lb=ROW_MAJOR, lc=ROW_MAJOR, ta=BF16, tc=None,
                 policy="auto", force_g=0, hybrid_min_waves=2, num_cus=0, occupancy=0, tile=None,
                 raster_rows=0, xcds=0, share="proportional", fixup="auto", spin_limit=0):
        self._h = ctypes.c_void_p()
        o = _options(policy, force_g, hybrid_min_waves, num_cus, occupancy, tile, raster_rows, xcds, share, fixup,
                     spin_limit)
        tc = ta if tc is None else tc
        _check(lib().skgemm_batched_plan(ctypes.byref(self._h), int(batch), int(M), int(N), int(K), la, lb, lc, ta,
                                         ta, tc, ctypes.byref(o)), "skgemm_batched_plan")
        self.batch, self.M, self.N, self.K = int(batch), int(M), int(N), int(K)
        self.la, self.lb, self.lc, self.ta, self.tc = la, lb, lc, ta, tc

    def batched_run(self, A, lda, sa, B, ldb, sb, C, ldc, sc, alpha=1.0, beta=0.0, scale_a=None, scale_b=None,
                    workspace=None, ws_bytes=0, stream=None, trace=None, trace_records=0):
        if trace is None:
            _check(lib().skgemm_batched_run(self._h, A, int(lda), int(sa), B, int(ldb), int(sb), C, int(ldc),
                                            int(sc), float(alpha), float(beta), scale_a, scale_b, workspace,
                                            int(ws_bytes), stream), "skgemm_batched_run")
        else:
            _check(lib().skgemm_batched_run_traced(self._h, A, int(lda), int(sa), B, int(ldb), int(sb), C,
                                                   int(ldc), int(sc), float(alpha), float(beta), scale_a, scale_b,
                                                   workspace, int(ws_bytes), trace, int(trace_records), stream),
                   "skgemm_batched_run_traced")


class ConvPlan(Plan):
    """Owns one implicit-GEMM convolution skgemm_plan_t (x NHWC, w KRSC, y NPQK)."""

    def __init__(self, n, h, w, c, k, r, s, pad=(0, 0), stride=(1, 1), dilation=(1, 1), ta=BF16, tc=None,
                 policy="auto", force_g=0, hybrid_min_waves=2, num_cus=0, occupancy=0, tile=None,
                 raster_rows=0, xcds=0, share="proportional", fixup="auto", spin_limit=0):
        self._h = ctypes.c_void_p()
        o = _options(policy, force_g, hybrid_min_waves, num_cus, occupancy, tile, raster_rows, xcds, share, fixup,
                     spin_limit)
        d = ConvDesc(int(n), int(h), int(w), int(c), int(k), int(r), int(s), int(pad[0]), int(pad[1]),
                     int(stride[0]), int(stride[1]), int(dilation[0]), int(dilation[1]))
        tc = ta if tc is None else tc
        _check(lib().skgemm_conv_plan(ctypes.byref(self._h), ctypes.byref(d), ta, tc, ctypes.byref(o)),
               "skgemm_conv_plan")
        self.desc = d
        self.ta, self.tc = ta, tc
        i = self.info()
        self.M, self.N, self.K = i["M"], i["N"], i["K"]

    def conv_run(self, x, w, y, alpha=1.0, beta=0.0, workspace=None, ws_bytes=0, stream=None, trace=None,
                 trace_records=0):
        if trace is None:
            _check(lib().skgemm_conv_run(self._h, x, w, y, float(alpha), float(beta), workspace, int(ws_bytes),
                                         stream), "skgemm_conv_run")
        else:
            _check(lib().skgemm_conv_run_traced(self._h, x, w, y, float(alpha), float(beta), workspace,
                                                int(ws_bytes), trace, int(trace_records), stream),
                   "skgemm_conv_run_traced")


def _options(policy, force_g, hybrid_min_waves, num_cus, occupancy, tile, raster_rows, xcds, share, fixup,
             spin_limit):
    o = default_options()
    if tile:
        o.tile_m, o.tile_n, o.tile_k = (int(x) for x in tile[:3])
        if len(tile) > 3:
            o.tile_waves = int(tile[3])
    o.raster_rows, o.xcds = int(raster_rows), int(xcds)
    o.share = SHARE[share] if isinstance(share, str) else int(share)
    o.fixup = FIXUP[fixup] if isinstance(fixup, str) else int(fixup)
    o.policy = POLICY[policy] if isinstance(policy, str) else int(policy)
    o.force_g = int(force_g)
    o.hybrid_min_waves = int(hybrid_min_waves)
    o.num_cus = int(num_cus)
    o.spin_limit = int(spin_limit)
    o.occupancy = int(occupancy)
    return o


class GroupedPlan(Plan):
    """Owns one grouped skgemm_plan_t (several problems, one launch)."""

    def __init__(self, Ms, Ns, Ks, la=ROW_MAJOR, lb=ROW_MAJOR, lc=ROW_MAJOR, ta=BF16, tc=None,
                 policy="auto", force_g=0, hybrid_min_waves=2, num_cus=0, occupancy=0, tile=None,
                 raster_rows=0, xcds=0, share="proportional", fixup="auto", spin_limit=0):
        self._h = ctypes.c_void_p()
        G = len(Ms)
        if not (len(Ns) == len(Ks) == G):
            raise ValueError("Ms, Ns, Ks must have the same length")
        o = default_options()
        if tile:
            o.tile_m, o.tile_n, o.tile_k = (int(x) for x in tile[:3])
            if len(tile) > 3:
                o.tile_waves = int(tile[3])
        o.raster_rows, o.xcds = int(raster_rows), int(xcds)
        o.share = SHARE[share] if isinstance(share, str) else int(share)
        o.fixup = FIXUP[fixup] if isinstance(fixup, str) else int(fixup)
        o.policy = POLICY[policy] if isinstance(policy, str) else int(policy)
        o.force_g = int(force_g)
        o.hybrid_min_waves = int(hybrid_min_waves)
        o.num_cus = int(num_cus)
        o.spin_limit = int(spin_limit)
        o.occupancy = int(occupancy)
        tc = ta if tc is None else tc
        arr = ctypes.c_int64 * max(G, 1)
        _check(lib().skgemm_grouped_plan(ctypes.byref(self._h), G, arr(*Ms), arr(*Ns), arr(*Ks), la, lb, lc, ta, ta,
                                         tc, ctypes.byref(o)), "skgemm_grouped_plan")
        self.Ms, self.Ns, self.Ks = [int(x) for x in Ms], [int(x) for x in Ns], [int(x) for x in Ks]
        self.la, self.lb, self.lc, self.ta, self.tc = la, lb, lc, ta, tc

    def table_size(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().skgemm_grouped_table_size(self._h, ctypes.byref(n)), "skgemm_grouped_table_size")
        return n.value

    def table(self, args) -> bytes:
        """Host table for args: list of (A, lda, B, ldb, C, ldc, alpha, beta) with device pointers."""
        G = len(self.Ms)
        ga = (GroupArgs * G)()
        for i, (A, lda, B, ldb, C, ldc, alpha, beta) in enumerate(args):
            ga[i] = GroupArgs(A, B, C, int(lda), int(ldb), int(ldc), float(alpha), float(beta))
        n = self.table_size()
        buf = ctypes.create_string_buffer(n)
        _check(lib().skgemm_grouped_table(self._h, ga, buf, n), "skgemm_grouped_table")
        return buf.raw

    def grouped_run(self, table_dev, workspace=None, ws_bytes=0, stream=None):
        _check(lib().skgemm_grouped_run(self._h, table_dev, workspace, int(ws_bytes), stream), "skgemm_grouped_run")

    def grouped_run_traced(self, table_dev, workspace, ws_bytes, trace, trace_records, stream=None):
        _check(lib().skgemm_grouped_run_traced(self._h, table_dev, workspace, int(ws_bytes), trace,
                                               int(trace_records), stream), "skgemm_grouped_run_traced")


def check_device_error(workspace_ptr, stream=None):
    _check(lib().skgemm_check_device_error(workspace_ptr, stream), "skgemm_check_device_error")


# ---------------------------------------------------------------- torch layer

_TORCH_DT = None


def _torch_dtypes():
    global _TORCH_DT
    if _TORCH_DT is None:
        import torch
        _TORCH_DT = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16,
                     torch.float8_e4m3fn: F8E4M3, torch.float64: F64}
    return _TORCH_DT


def _layouts(t):
    """Every valid (layout, ld) reading of a 2-D tensor's strides (a tensor with
    a dimension of size <= 1 is both row- and column-major)."""
    r, c = t.shape
    if t.numel() == 0:          # no element is addressed: any reading is valid
        return [(ROW_MAJOR, max(c, 1)), (COL_MAJOR, max(r, 1))]
    s0, s1 = t.stride()
    out = []
    if s1 == 1 or c <= 1:
        out.append((ROW_MAJOR, max(s0, c, 1)))
    if s0 == 1 or r <= 1:
        out.append((COL_MAJOR, max(s1, r, 1)))
    return out


def _layout(t, prefer=ROW_MAJOR):
    """(layout, ld) of a 2-D tensor, the preferred reading when both are valid,
    or None if neither dimension is contiguous."""
    ls = _layouts(t)
    for lay in ls:
        if lay[0] == prefer:
            return lay
    return ls[0] if ls else None


def _pick(tensors, prefer):
    """One layout valid for every tensor of a group (the preferred one if
    possible), with each tensor's leading dimension; None if there is none."""
    common = {ROW_MAJOR, COL_MAJOR}
    for t in tensors:
        common &= {lay for lay, _ in _layouts(t)}
    if not common:
        return None
    lay = prefer if prefer in common else common.pop()
    return lay, [dict(_layouts(t))[lay] for t in tensors]


_ws_cache = {}      # (device index, stream handle) -> zero-filled workspace tensor
_ws_retired = []    # replaced workspaces, kept alive: a captured graph may still use them
_plan_cache = {}
_check_runs = False


def workspace(nbytes: int, device, stream=None):
    """A zero-filled, 256-byte aligned device workspace of at least nbytes for
    runs on `stream` (a hipStream_t handle; None = the device's current
    stream).  One per (device, stream): runs on one stream are ordered, so
    they may share it, while runs on different streams each get their own.
    A workspace that is outgrown is replaced and the old one is kept alive
    until the process ends (a HIP graph captured earlier may still hold its
    address)."""
    import torch
    dev = device if isinstance(device, torch.device) else torch.device(device)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev.index, int(stream or 0))
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        if buf is not None:
            _ws_retired.append(buf)
        with torch.cuda.stream(torch.cuda.ExternalStream(stream, device=dev)) if stream else \
                torch.cuda.device(dev):
            buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
        _ws_cache[key] = buf
    return buf


def set_error_checks(on: bool) -> None:
    """When on, matmul and grouped_matmul synchronise their stream after each
    launch and read the workspace's error word (check_workspace)."""
    global _check_runs
    _check_runs = bool(on)


def check_workspace(ws, stream=None) -> None:
    """Raise SkgemmError(ERR_TIMEOUT) if a fix-up wait of a run on workspace
    tensor `ws` expired (synchronises `stream`).  The workspace is zero-filled
    again first, so the next run on it starts from clear flags."""
    st = lib().skgemm_check_device_error(ws.data_ptr(), stream)
    if st == ERR_TIMEOUT:
        ws.zero_()
        import torch
        torch.cuda.synchronize(ws.device)
    _check(st, "skgemm_check_device_error")


def check_device_errors() -> None:
    """Check every cached workspace (see check_workspace); raises on the first
    one whose error word is set, after clearing it."""
    for (_, stream), ws in list(_ws_cache.items()):
        check_workspace(ws, stream or None)


def get_plan(M, N, K, la, lb, lc, ta, tc, policy="auto", force_g=0, hybrid_min_waves=2, tile=None, fixup="auto",
             spin_limit=0):
    key = (M, N, K, la, lb, lc, ta, tc, policy, force_g, hybrid_min_waves, tuple(tile) if tile else None, fixup,
           spin_limit)
    p = _plan_cache.get(key)
    if p is None:
        p = Plan(M, N, K, la, lb, lc, ta, tc, policy=policy, force_g=force_g, hybrid_min_waves=hybrid_min_waves,
                 tile=tile, fixup=fixup, spin_limit=spin_limit)
        if len(_plan_cache) > 4096:
            _plan_cache.clear()
        _plan_cache[key] = p
    return p


def matmul(A, B, out=None, *, out_dtype=None, alpha=1.0, beta=0.0, scale_a=None, scale_b=None,
           policy="auto", force_g=0, hybrid_min_waves=2, trace=None, tile=None, fixup="auto", spin_limit=0,
           check=None, times=None):
    """C = alpha * s_A * s_B * A @ B + beta * C on torch tensors (2-D, on one GPU).

    Layouts come from the strides (a non-contiguous operand is copied).  When
    ``out`` is given it receives the result and supplies C for beta != 0.
    ``trace``, when given, is an int32 device tensor of at least
    8 * plan.trace_capacity() elements that receives the schedule records;
    ``times`` (int64, 7 per record) adds each segment's timestamps and shader-clock counts.
    ``check`` (default: set_error_checks) synchronises after the launch and
    raises SkgemmError(ERR_TIMEOUT), with the workspace cleared, if a fix-up
    wait expired."""
    import torch
    fast = (out is None and trace is None and scale_a is None and scale_b is None and beta == 0.0
            and not (check or (check is None and _check_runs)))
    if fast:
        key = (A.shape, A.stride(), B.shape, B.stride(), A.dtype, B.dtype, A.device, out_dtype, policy, force_g,
               hybrid_min_waves, tuple(tile) if tile else None, fixup, spin_limit)
        ent = _fast_cache.get(key)
        if ent is not None:
            return _fast_run(ent, A, B, alpha)
    dts = _torch_dtypes()
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("matmul needs A (M x K) and B (K x N)")
    if A.dtype != B.dtype or A.dtype not in dts:
        raise ValueError(f"unsupported input dtypes {A.dtype}, {B.dtype}")
    if not A.is_cuda or A.device != B.device:
        raise ValueError("operands must live on the same GPU")
    M, K = A.shape
    N = B.shape[1]
    # where a degenerate shape allows either reading, take the K-contiguous one
    la = _layout(A, prefer=ROW_MAJOR)
    if la is None:
        A = A.contiguous()
        la = _layout(A)
        fast = False          # the layout is the copy's, not the caller's tensor's
    lb = _layout(B, prefer=COL_MAJOR)
    if lb is None:
        B = B.contiguous()
        lb = _layout(B)
        fast = False
    if out is None:
        if out_dtype is None:
            out_dtype = torch.float32 if A.dtype in (torch.float32, torch.float8_e4m3fn) else A.dtype
        out = torch.empty((M, N), dtype=out_dtype, device=A.device)
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
    lc = _layout(out)
    if lc is None or out.shape != (M, N):
        raise ValueError("out must be an M x N tensor with one contiguous dimension")
    plan = get_plan(M, N, K, la[0], lb[0], lc[0], dts[A.dtype], dts[out.dtype], policy, force_g, hybrid_min_waves,
                    tile, fixup, spin_limit)
    nws = plan.workspace_size()
    stream = torch.cuda.current_stream(A.device).cuda_stream
    ws = workspace(nws, A.device, stream) if nws else None
    args = (A.data_ptr() if A.numel() else None, la[1], B.data_ptr() if B.numel() else None, lb[1],
            out.data_ptr() if out.numel() else None, lc[1], alpha, beta,
            scale_a.data_ptr() if scale_a is not None else None,
            scale_b.data_ptr() if scale_b is not None else None,
            ws.data_ptr() if ws is not None else None, nws)
    if trace is None:
        plan.run(*args, stream=stream)
    elif times is None:
        plan.run_traced(*args, trace.data_ptr(), trace.numel() // 8, stream=stream)
    else:
        n = min(trace.numel() // 8, times.numel() // 7)
        plan.run_timed(*args, trace.data_ptr(), times.data_ptr(), n, stream=stream)
    if ws is not None and (_check_runs if check is None else check):
        check_workspace(ws, stream)
    if fast and M * N * K > 0 and len(_fast_cache) < 4096:
        # everything this call derived from the tensors' shapes, strides and
        # types, for the next call with the same signature
        _fast_cache[key] = (lib().skgemm_run, plan.handle, la[1], lb[1], lc[1], nws, M, N, out.dtype, A.device,
                            plan)
    return out


_fast_cache = {}


def _raw_stream(device):
    """hipStream_t of the device's current stream (torch's raw accessor when it
    has one: it skips building a Stream object)."""
    import torch
    get = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if get is not None:
        return get(device.index)
    return torch.cuda.current_stream(device).cuda_stream


def _fast_run(ent, A, B, alpha):
    """matmul for a signature seen before: no layout inference, no plan lookup."""
    import torch
    fn, handle, lda, ldb, ldc, nws, M, N, odt, dev, _plan = ent
    out = torch.empty((M, N), dtype=odt, device=dev)
    stream = _raw_stream(dev)
    wsp = None
    if nws:
        ws = _ws_cache.get((dev.index, int(stream or 0)))
        if ws is None or ws.numel() < nws:
            ws = workspace(nws, dev, stream)
        wsp = ws.data_ptr()
    st = fn(handle, A.data_ptr(), lda, B.data_ptr(), ldb, out.data_ptr(), ldc, float(alpha), 0.0, None, None, wsp,
            nws, stream)
    if st != OK:
        raise SkgemmError(st, "skgemm_run")
    return out


def _layout_of(t):
    la = _layout(t)
    if la is None:
        raise ValueError("operand needs one contiguous dimension")
    return la


_gplan_cache = {}


def grouped_matmul(As, Bs, Cs=None, *, out_dtype=None, alpha=1.0, beta=0.0, policy="auto", force_g=0,
                   hybrid_min_waves=2, trace=None, table=None, tile=None, spin_limit=0, check=None):
    """C_i = alpha * A_i @ B_i + beta * C_i for every i, in ONE persistent launch.

    All A_i share a layout, all B_i share a layout, all C_i share a layout
    and every tensor the same dtype pair.  Returns (Cs, table) where table is
    the device tensor of the per-problem descriptors; passing it back in with
    the same tensors skips rebuilding it (e.g. for graph capture)."""
    import torch
    dts = _torch_dtypes()
    G = len(As)
    if G == 0 or len(Bs) != G:
        raise ValueError("need as many A as B")
    dev = As[0].device
    if out_dtype is None:
        out_dtype = torch.float32 if As[0].dtype in (torch.float32, torch.float8_e4m3fn) else As[0].dtype
    if Cs is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs Cs")
        Cs = [torch.empty((A.shape[0], B.shape[1]), dtype=out_dtype, device=dev) for A, B in zip(As, Bs)]
    pa, pb, pc = _pick(As, ROW_MAJOR), _pick(Bs, COL_MAJOR), _pick(Cs, ROW_MAJOR)
    if pa is None or pb is None or pc is None:
        raise ValueError("all A (B, C) of a group must share one layout")
    (la, lda), (lb, ldb), (lc, ldc) = pa, pb, pc
    Ms = [A.shape[0] for A in As]
    Ns = [B.shape[1] for B in Bs]
    Ks = [A.shape[1] for A in As]
    key = (tuple(Ms), tuple(Ns), tuple(Ks), la, lb, lc, dts[As[0].dtype], dts[Cs[0].dtype], policy, force_g,
           hybrid_min_waves, tuple(tile) if tile else None, spin_limit)
    plan = _gplan_cache.get(key)
    if plan is None:
        plan = GroupedPlan(Ms, Ns, Ks, la, lb, lc, dts[As[0].dtype], dts[Cs[0].dtype], policy=policy,
                           force_g=force_g, hybrid_min_waves=hybrid_min_waves, tile=tile, spin_limit=spin_limit)
        if len(_gplan_cache) > 256:
            _gplan_cache.clear()
        _gplan_cache[key] = plan
    if table is None:
        args = []
        for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
            args.append((A.data_ptr() if A.numel() else None, lda[i],
                         B.data_ptr() if B.numel() else None, ldb[i],
                         C.data_ptr() if C.numel() else None, ldc[i], alpha, beta))
        host = plan.table(args)
        table = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(dev)
    nws = plan.workspace_size()
    stream = torch.cuda.current_stream(dev).cuda_stream
    ws = workspace(nws, dev, stream) if nws else None
    if trace is None:
        plan.grouped_run(table.data_ptr(), ws.data_ptr() if ws is not None else None, nws, stream)
    else:
        plan.grouped_run_traced(table.data_ptr(), ws.data_ptr() if ws is not None else None, nws,
                                trace.data_ptr(), trace.numel() // 8, stream)
    if ws is not None and (_check_runs if check is None else check):
        check_workspace(ws, stream)
    return Cs, table


_bplan_cache = {}


def _layout3(t, prefer):
    """(layout, ld, batch stride) of a 3-D tensor whose matrices have one
    contiguous dimension, or None."""
    lay = _layout(t[0] if t.shape[0] else t.new_empty(t.shape[1:]), prefer)
    if t.shape[0] == 0 or lay is None:
        return None
    if t.shape[1] * t.shape[2] and t.shape[0] > 1:
        # every matrix has the same strides as the first
        s0, s1, s2 = t.stride()
        m = t[0]
        if m.stride() != (s1, s2):
            return None
    return lay[0], lay[1], t.stride(0)


def batched_matmul(A, B, out=None, *, out_dtype=None, alpha=1.0, beta=0.0, policy="auto", force_g=0,
                   hybrid_min_waves=2, tile=None, trace=None):
    """C[i] = alpha * A[i] @ B[i] + beta * C[i] for 3-D tensors (batch, M, K) and
    (batch, K, N) in one persistent launch (strided batched Stream-K GEMM)."""
    import torch
    dts = _torch_dtypes()
    if A.dim() != 3 or B.dim() != 3 or A.shape[0] != B.shape[0] or A.shape[2] != B.shape[1]:
        raise ValueError("batched_matmul needs A (batch x M x K) and B (batch x K x N)")
    if A.dtype != B.dtype or A.dtype not in dts:
        raise ValueError(f"unsupported input dtypes {A.dtype}, {B.dtype}")
    batch, M, K = A.shape
    N = B.shape[2]
    la = _layout3(A, ROW_MAJOR)
    if la is None:
        A = A.contiguous()
        la = _layout3(A, ROW_MAJOR)
    lb = _layout3(B, COL_MAJOR)
    if lb is None:
        B = B.contiguous()
        lb = _layout3(B, COL_MAJOR)
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        if out_dtype is None:
            out_dtype = torch.float32 if A.dtype in (torch.float32, torch.float8_e4m3fn) else A.dtype
        out = torch.empty((batch, M, N), dtype=out_dtype, device=A.device)
    lc = _layout3(out, ROW_MAJOR)
    if lc is None or tuple(out.shape) != (batch, M, N):
        raise ValueError("out must be batch x M x N with one contiguous dimension per matrix")
    key = (batch, M, N, K, la[0], lb[0], lc[0], dts[A.dtype], dts[out.dtype], policy, force_g, hybrid_min_waves,
           tuple(tile) if tile else None)
    plan = _bplan_cache.get(key)
    if plan is None:
        plan = BatchedPlan(batch, M, N, K, la[0], lb[0], lc[0], dts[A.dtype], dts[out.dtype], policy=policy,
                           force_g=force_g, hybrid_min_waves=hybrid_min_waves, tile=tile)
        if len(_bplan_cache) > 256:
            _bplan_cache.clear()
        _bplan_cache[key] = plan
    nws = plan.workspace_size()
    stream = torch.cuda.current_stream(A.device).cuda_stream
    ws = workspace(nws, A.device, stream) if nws else None
    plan.batched_run(A.data_ptr() if A.numel() else None, la[1], la[2], B.data_ptr() if B.numel() else None, lb[1],
                     lb[2], out.data_ptr() if out.numel() else None, lc[1], lc[2], alpha, beta,
                     workspace=ws.data_ptr() if ws is not None else None, ws_bytes=nws, stream=stream,
                     trace=trace.data_ptr() if trace is not None else None,
                     trace_records=trace.numel() // 8 if trace is not None else 0)
    if ws is not None and _check_runs:
        check_workspace(ws, stream)
    return out


_cplan_cache = {}


def conv2d(x, w, out=None, *, padding=(0, 0), stride=(1, 1), dilation=(1, 1), out_dtype=None, alpha=1.0,
           beta=0.0, policy="auto", force_g=0, hybrid_min_waves=2, tile=None, trace=None):
    """y = alpha * conv2d(x, w) + beta * y as one Stream-K implicit-GEMM launch.

    x is (N, H, W, C) and w is (K, R, S, C), both channels-last and contiguous,
    in bfloat16 or float16 with C a multiple of 64; the result is (N, P, Q, K)
    (cross-correlation, zero padding), in the input type or float32."""
    import torch
    dts = _torch_dtypes()
    if x.dim() != 4 or w.dim() != 4 or x.shape[3] != w.shape[3]:
        raise ValueError("conv2d needs x (N, H, W, C) and w (K, R, S, C)")
    if x.dtype != w.dtype or x.dtype not in (torch.bfloat16, torch.float16):
        raise ValueError(f"unsupported input dtypes {x.dtype}, {w.dtype}")
    if not x.is_contiguous() or not w.is_contiguous():
        raise ValueError("conv2d needs contiguous channels-last x and w")
    pad, std, dil = tuple(padding), tuple(stride), tuple(dilation)
    n, h, wd, c = x.shape
    k, r, s, _ = w.shape
    if out_dtype is None:
        out_dtype = out.dtype if out is not None else x.dtype
    key = (n, h, wd, c, k, r, s, pad, std, dil, dts[x.dtype], dts[out_dtype], policy, force_g, hybrid_min_waves,
           tuple(tile) if tile else None)
    plan = _cplan_cache.get(key)
    if plan is None:
        plan = ConvPlan(n, h, wd, c, k, r, s, pad, std, dil, dts[x.dtype], dts[out_dtype], policy=policy,
                        force_g=force_g, hybrid_min_waves=hybrid_min_waves, tile=tile)
        if len(_cplan_cache) > 256:
            _cplan_cache.clear()
        _cplan_cache[key] = plan
    P = (h + 2 * pad[0] - dil[0] * (r - 1) - 1) // std[0] + 1
    Q = (wd + 2 * pad[1] - dil[1] * (s - 1) - 1) // std[1] + 1
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((n, P, Q, k), dtype=out_dtype, device=x.device)
    elif tuple(out.shape) != (n, P, Q, k) or not out.is_contiguous() or out.dtype != out_dtype:
        raise ValueError(f"out must be a contiguous ({n}, {P}, {Q}, {k}) {out_dtype} tensor")
    nws = plan.workspace_size()
    stream = torch.cuda.current_stream(x.device).cuda_stream
    ws = workspace(nws, x.device, stream) if nws else None
    plan.conv_run(x.data_ptr() if x.numel() else None, w.data_ptr() if w.numel() else None,
                  out.data_ptr() if out.numel() else None, alpha, beta,
                  workspace=ws.data_ptr() if ws is not None else None, ws_bytes=nws, stream=stream,
                  trace=trace.data_ptr() if trace is not None else None,
                  trace_records=trace.numel() // 8 if trace is not None else 0)
    if ws is not None and _check_runs:
        check_workspace(ws, stream)
    return out


_qws = {}


def quantize_e4m3(X, layout="row", out=None, scale=None):
    """Per-tensor E4M3 quantisation of a 2-D FP32/BF16/FP16 tensor on the GPU.

    Returns (Q, scale): Q a float8_e4m3fn tensor of X's shape stored row-major
    (layout="row") or column-major (layout="col", a transposed view of an
    N x M row-major buffer), scale a 1-element FP32 device tensor."""
    import torch
    dts = _torch_dtypes()
    if X.dim() != 2 or X.dtype not in (torch.float32, torch.bfloat16, torch.float16):
        raise ValueError("quantize_e4m3 needs a 2-D FP32, BF16 or FP16 tensor")
    rows, cols = X.shape
    lx = _layout(X)
    if lx is None:
        X = X.contiguous()
        lx = _layout(X)
    if out is None:
        if layout == "row":
            out = torch.empty((rows, cols), dtype=torch.float8_e4m3fn, device=X.device)
        else:
            out = torch.empty((cols, rows), dtype=torch.float8_e4m3fn, device=X.device).t()
    lq = _layout(out, prefer=COL_MAJOR if layout == "col" else ROW_MAJOR)
    if lq is None:
        raise ValueError("out needs one contiguous dimension")
    if scale is None:
        scale = torch.empty(1, dtype=torch.float32, device=X.device)
    key = X.device.index
    ws = _qws.get(key)
    if ws is None:
        n = ctypes.c_size_t()
        _check(lib().skgemm_quantize_workspace_size(ctypes.byref(n)), "skgemm_quantize_workspace_size")
        ws = torch.empty(n.value // 4, dtype=torch.float32, device=X.device)
        _qws[key] = ws
    stream = torch.cuda.current_stream(X.device).cuda_stream
    _check(lib().skgemm_quantize_e4m3(X.data_ptr() if X.numel() else None, dts[X.dtype], rows, cols, lx[0], lx[1],
                                      out.data_ptr() if out.numel() else None, lq[0], lq[1], scale.data_ptr(),
                                      ws.data_ptr(), ws.numel() * 4, stream), "skgemm_quantize_e4m3")
    return out, scale


def matmul_fp8(A, B, *, out_dtype=None, alpha=1.0, policy="auto", force_g=0, tile=None):
    """FP8 GEMM of higher-precision A and B: per-tensor E4M3 quantisation of
    A (row-major) and B (column-major), then the FP8 Stream-K GEMM with the
    scales applied in the epilogue.  Returns (C, (qA, sA), (qB, sB))."""
    import torch
    qa, sa = quantize_e4m3(A, "row")
    qb, sb = quantize_e4m3(B, "col")
    C = matmul(qa, qb, out_dtype=out_dtype or torch.float32, alpha=alpha, scale_a=sa, scale_b=sb,
               policy=policy, force_g=force_g, tile=tile)
    return C, (qa, sa), (qb, sb)
