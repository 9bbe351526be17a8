"""Python binding of libsptrsv.so (ctypes). Argument marshalling only: every
step of the solve, the analysis and the rewrite runs in the library's HIP
kernels. torch supplies device memory (CUDA tensors on ROCm) and the stream.

Names mirror the C ABI in include/sptrsv.h.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsptrsv.so")

ORIGINAL, REWRITTEN, BATCH = 0, 1, 2
THIN_ROWS, THIN_COST = 0, 1
LOWER, UPPER, LOWER_TRANS, UPPER_TRANS = 0, 1, 2, 3  # triangular forms (sptrsv_analyze_form)
MLP_NIN = 20
MLP_NPARAM = 5569

STATUS_NAMES = ["OK", "ARG", "STATE", "NOT_LOWER", "UNSORTED", "MISSING_DIAG", "ZERO_PIVOT", "NONFINITE",
                "OVERFLOW", "ALLOC", "HIP", "TIMEOUT"]

EXPORTS = [
    "sptrsv_create", "sptrsv_destroy", "sptrsv_last_error", "sptrsv_status_name", "sptrsv_analyze", "sptrsv_analyze_form",
    "sptrsv_get_levels", "sptrsv_level_stats", "sptrsv_rewrite", "sptrsv_get_rewritten", "sptrsv_get_targets",
    "sptrsv_solve", "sptrsv_prepare", "sptrsv_check", "sptrsv_set_schedule", "sptrsv_get_schedule",
    "sptrsv_autotune", "sptrsv_autotune_rows", "sptrsv_graph_create", "sptrsv_graph_launch", "sptrsv_residual", "sptrsv_batch_analyze",
    "sptrsv_batch_solve", "sptrsv_batch_solve_looped", "sptrsv_batch_levels", "sptrsv_plan_save",
    "sptrsv_plan_load", "sptrsv_level_features", "sptrsv_mlp_forward", "sptrsv_mlp_backward", "sptrsv_mlp_adam",
    "sptrsv_mlp_mask", "sptrsv_profile", "sptrsv_level_times", "sptrsv_get_tune_info",
    "sptrsv_solve_noalloc", "sptrsv_measure_level_costs", "sptrsv_level_floor",
    "sptrsv_get_info", "sptrsv_level_finish_times", "sptrsv_mlp_actions", "sptrsv_solve_rows",
    "sptrsv_graph_create_rows",
]


class SptrsvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        self.name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{self.name}: {msg}")


class RewriteOpts(C.Structure):
    _fields_ = [("thin_metric", C.c_int32), ("thin_threshold", C.c_double), ("fill_cap", C.c_double),
                ("max_distance", C.c_int32), ("d_level_mask", C.c_void_p), ("max_indegree", C.c_int32),
                ("critical_only", C.c_int32), ("max_spread", C.c_int64), ("scan_workers", C.c_int32),
                ("d_level_budget", C.c_void_p), ("d_level_fill_cap", C.c_void_p), ("self_check", C.c_double)]


class RewriteStats(C.Structure):
    _fields_ = [("nlev_before", C.c_int32), ("nlev_after", C.c_int32), ("rows_rewritten", C.c_int32),
                ("max_distance", C.c_int32), ("target_steps", C.c_int32), ("nnz_L", C.c_int64),
                ("nnz_Lp", C.c_int64), ("nnz_T", C.c_int64), ("total_cost_before", C.c_int64),
                ("total_cost_after", C.c_int64), ("avg_level_cost_before", C.c_double),
                ("avg_level_cost_after", C.c_double), ("rows_skipped", C.c_int32),
                ("self_check_failed", C.c_int32), ("self_check_err", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double)]


PROFILE_CLASSES = ["gather", "thin_run", "wide_level", "scatter"]


class TuneInfo(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("timed_out", C.c_int32), ("best_ms", C.c_float),
                ("max_wait_limit_ms", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("form", C.c_int32), ("n", C.c_int32), ("nlev", C.c_int32), ("has_rewrite", C.c_int32),
                ("nnz", C.c_int64)]


class LevelCosts(C.Structure):
    _fields_ = [("thin_level_ns", C.c_double), ("thin_wave_level_ns", C.c_double), ("launch_ns", C.c_double),
                ("graph_node_ns", C.c_double), ("grid_barrier_ns", C.c_double), ("flag_hop_ns", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Schedule(C.Structure):
    _fields_ = [("mode", C.c_int32), ("thin_rows", C.c_int32), ("wg_threads", C.c_int32),
                ("wide_threads", C.c_int32), ("lanes_per_row", C.c_int32), ("wide_grid", C.c_int32),
                ("overlap", C.c_int32), ("thin_cols", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libsptrsv.so; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_05843_amd.build` "
                           "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
    sig = {
        "sptrsv_create": [C.POINTER(vp)],
        "sptrsv_destroy": [vp],
        "sptrsv_analyze": [vp, i32, i32, vp, vp, vp, vp, C.POINTER(i32)],
        "sptrsv_analyze_form": [vp, i32, i32, i32, vp, vp, vp, vp, C.POINTER(i32)],
        "sptrsv_get_levels": [vp, C.c_int, vp, vp, vp, vp],
        "sptrsv_level_stats": [vp, C.c_int, vp, vp, vp, C.POINTER(i64), C.POINTER(dbl), vp],
        "sptrsv_rewrite": [vp, C.POINTER(RewriteOpts), vp, C.POINTER(RewriteStats)],
        "sptrsv_get_rewritten": [vp, vp, vp, vp, vp, vp, vp, vp],
        "sptrsv_get_targets": [vp, vp, vp],
        "sptrsv_solve": [vp, C.c_int, i32, vp, i64, vp, i64, vp],
        "sptrsv_solve_noalloc": [vp, C.c_int, i32, vp, i64, vp, i64, vp],
        "sptrsv_solve_rows": [vp, C.c_int, i32, vp, vp, vp],
        "sptrsv_graph_create_rows": [vp, C.c_int, i32, vp, vp, vp, C.POINTER(i32)],
        "sptrsv_prepare": [vp, C.c_int, i32, vp],
        "sptrsv_check": [vp, vp],
        "sptrsv_set_schedule": [vp, C.c_int, C.POINTER(Schedule)],
        "sptrsv_get_schedule": [vp, C.c_int, C.c_int32, C.POINTER(Schedule)],
        "sptrsv_autotune": [vp, C.c_int, i32, vp, C.POINTER(f32)],
        "sptrsv_autotune_rows": [vp, C.c_int, i32, vp, C.POINTER(f32)],
        "sptrsv_graph_create": [vp, C.c_int, i32, vp, i64, vp, i64, vp, C.POINTER(i32)],
        "sptrsv_graph_launch": [vp, i32, vp],
        "sptrsv_residual": [vp, i32, vp, i64, vp, i64, C.POINTER(dbl), vp],
        "sptrsv_batch_analyze": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
        "sptrsv_batch_solve": [vp, i32, vp, vp, vp],
        "sptrsv_batch_solve_looped": [vp, i32, vp, vp, vp],
        "sptrsv_batch_levels": [vp, i32, C.POINTER(i32), vp, vp, vp],
        "sptrsv_plan_save": [vp, C.c_char_p],
        "sptrsv_plan_load": [vp, C.c_char_p],
        "sptrsv_level_features": [vp, vp, vp],
        "sptrsv_mlp_forward": [vp, vp, vp, i32, vp, vp],
        "sptrsv_mlp_backward": [vp, vp, vp, vp, vp, i32, vp, vp, vp],
        "sptrsv_level_times": [vp, C.c_int, i32, vp, vp, vp],
        "sptrsv_mlp_adam": [vp, vp, vp, vp, i32, f32, vp],
        "sptrsv_mlp_mask": [vp, i32, f32, vp, vp],
        "sptrsv_mlp_actions": [vp, i32, i32, C.POINTER(f32), C.POINTER(i32), C.POINTER(f32), vp, vp, vp, vp],
        "sptrsv_level_finish_times": [vp, C.c_int, i32, vp, vp, vp],
        "sptrsv_profile": [vp, C.c_int, vp, vp],
        "sptrsv_get_tune_info": [vp, C.POINTER(TuneInfo)],
        "sptrsv_measure_level_costs": [vp, vp, C.POINTER(LevelCosts)],
        "sptrsv_level_floor": [vp, C.c_int, i32, i32, C.POINTER(LevelCosts), C.POINTER(dbl)],
        "sptrsv_get_info": [vp, C.POINTER(Info), C.POINTER(RewriteStats)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.sptrsv_last_error.argtypes = [vp]
    L.sptrsv_last_error.restype = C.c_char_p
    L.sptrsv_status_name.argtypes = [C.c_int]
    L.sptrsv_status_name.restype = C.c_char_p
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda, "device tensor expected"
    return t.data_ptr()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(cond, msg):
    if not cond:
        raise ValueError(msg)


def _check_free(st: int, msg: str = ""):
    if st != 0:
        raise SptrsvError(st, msg)


def mlp_forward(params, feat, norm=None, prob=None):
    B = feat.shape[0]
    prob = prob if prob is not None else torch.empty(B, dtype=torch.float32, device=feat.device)
    _check_free(lib().sptrsv_mlp_forward(_ptr(params), _ptr(feat), _ptr(norm), B, _ptr(prob), _stream()),
                "mlp_forward")
    return prob


def mlp_backward(params, feat, label, weight=None, norm=None):
    B = feat.shape[0]
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    _check_free(lib().sptrsv_mlp_backward(_ptr(params), _ptr(feat), _ptr(norm), _ptr(label), _ptr(weight), B,
                                          _ptr(grad), _ptr(loss), _stream()), "mlp_backward")
    return grad, loss


def mlp_adam(params, grad, m, v, step: int, lr: float):
    _check_free(lib().sptrsv_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, _stream()), "mlp_adam")


def mlp_mask(prob, threshold: float = 0.5):
    mask = torch.empty(prob.shape[0], dtype=torch.uint8, device=prob.device)
    _check_free(lib().sptrsv_mlp_mask(_ptr(prob), prob.shape[0], threshold, _ptr(mask), _stream()), "mlp_mask")
    return mask


MAX_TIERS = 4


def mlp_actions(prob, tiers):
    """Tiered actions from probabilities: tiers = [(threshold, budget, cap),
    ...] with ascending thresholds; returns the (mask, budget, cap) device
    arrays for Handle.rewrite(mask, level_budget=, level_fill_cap=)."""
    k = len(tiers)
    nlev = prob.shape[0]
    thr = (C.c_float * max(k, 1))(*[float(t[0]) for t in tiers])
    bud = (C.c_int32 * max(k, 1))(*[int(t[1]) for t in tiers])
    cap = (C.c_float * max(k, 1))(*[float(t[2]) for t in tiers])
    mask = torch.empty(nlev, dtype=torch.uint8, device=prob.device)
    budget = torch.empty(nlev, dtype=torch.int32, device=prob.device)
    fcap = torch.empty(nlev, dtype=torch.float32, device=prob.device)
    _check_free(lib().sptrsv_mlp_actions(_ptr(prob), nlev, k, thr, bud, cap, _ptr(mask), _ptr(budget), _ptr(fcap),
                                         _stream()), "mlp_actions")
    return mask, budget, fcap


class Handle:
    """One analysed matrix (plus its rewrite and batched matrices)."""

    def __init__(self):
        self._L = lib()
        h = C.c_void_p()
        st = self._L.sptrsv_create(C.byref(h))
        if st != 0:
            raise SptrsvError(st, "sptrsv_create failed")
        self._h = h
        self.n = 0
        self.nlev = 0
        self.rstats = None
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._L.sptrsv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise SptrsvError(st, self._L.sptrsv_last_error(self._h).decode())

    # ------------------------------------------------------------------ analysis
    def analyze(self, row_ptr, col, val, form=LOWER) -> int:
        """form: LOWER (L x = b), UPPER (U x = b), LOWER_TRANS (L^T x = b, given
        L) or UPPER_TRANS (U^T x = b, given U); solves take and return b, x in
        the caller's numbering."""
        _need(row_ptr.dtype == torch.int32 and col.dtype == torch.int32 and val.dtype == torch.float64,
              "int32 row_ptr/col and float64 val expected")
        n = row_ptr.numel() - 1
        nnz = col.numel()
        nl = C.c_int32(0)
        self._check(self._L.sptrsv_analyze_form(self._h, int(form), n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val),
                                                _stream(), C.byref(nl)))
        self.n, self.nlev, self.rstats = n, nl.value, None
        return nl.value

    def levels(self, which=ORIGINAL):
        nlev = self.nlev if which == ORIGINAL else self.rstats["nlev_after"]
        dev = torch.device("cuda")
        lp = torch.empty(nlev + 1, dtype=torch.int32, device=dev)
        lr = torch.empty(self.n, dtype=torch.int32, device=dev)
        rl = torch.empty(self.n, dtype=torch.int32, device=dev)
        self._check(self._L.sptrsv_get_levels(self._h, which, _ptr(lp), _ptr(lr), _ptr(rl), _stream()))
        return lp, lr, rl

    def level_stats(self, which=ORIGINAL):
        nlev = self.nlev if which == ORIGINAL else self.rstats["nlev_after"]
        dev = torch.device("cuda")
        rows, nnz, cost = (torch.empty(nlev, dtype=torch.int64, device=dev) for _ in range(3))
        tot, avg = C.c_int64(0), C.c_double(0)
        self._check(self._L.sptrsv_level_stats(self._h, which, _ptr(rows), _ptr(nnz), _ptr(cost), C.byref(tot),
                                               C.byref(avg), _stream()))
        return dict(rows=rows, nnz=nnz, cost=cost, total=tot.value, avg=avg.value)

    # ------------------------------------------------------------------- rewrite
    def rewrite(self, thin_metric=THIN_ROWS, thin_threshold=32.0, fill_cap=4.0, max_distance=0, mask=None,
                max_indegree=0, max_spread=0, critical_only=False, scan_workers=1, self_check=0.0,
                level_budget=None, level_fill_cap=None):
        if mask is not None:
            _need(mask.dtype == torch.uint8 and mask.numel() >= self.nlev, "uint8 mask of nlev entries expected")
        if level_budget is not None:
            _need(level_budget.dtype == torch.int32 and level_budget.numel() >= self.nlev,
                  "int32 level_budget of nlev entries expected")
        if level_fill_cap is not None:
            _need(level_fill_cap.dtype == torch.float32 and level_fill_cap.numel() >= self.nlev,
                  "float32 level_fill_cap of nlev entries expected")
        o = RewriteOpts(thin_metric, float(thin_threshold), float(fill_cap), int(max_distance),
                        _ptr(mask) if mask is not None else None, int(max_indegree), int(bool(critical_only)),
                        int(max_spread), int(scan_workers), _ptr(level_budget), _ptr(level_fill_cap),
                        float(self_check))
        st = RewriteStats()
        self._check(self._L.sptrsv_rewrite(self._h, C.byref(o), _stream(), C.byref(st)))
        self.rstats = st.as_dict()
        return self.rstats

    def rewritten(self):
        s = self.rstats
        dev = torch.device("cuda")
        out = dict(lp_ptr=torch.empty(self.n + 1, dtype=torch.int32, device=dev),
                   lp_col=torch.empty(s["nnz_Lp"], dtype=torch.int32, device=dev),
                   lp_val=torch.empty(s["nnz_Lp"], dtype=torch.float64, device=dev),
                   t_ptr=torch.empty(self.n + 1, dtype=torch.int32, device=dev),
                   t_col=torch.empty(s["nnz_T"], dtype=torch.int32, device=dev),
                   t_val=torch.empty(s["nnz_T"], dtype=torch.float64, device=dev))
        self._check(self._L.sptrsv_get_rewritten(self._h, *[_ptr(out[k]) for k in
                                                            ["lp_ptr", "lp_col", "lp_val", "t_ptr", "t_col",
                                                             "t_val"]], _stream()))
        return out

    def targets(self):
        t = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self._check(self._L.sptrsv_get_targets(self._h, _ptr(t), _stream()))
        return t

    # --------------------------------------------------------------------- solve
    def solve(self, b, which=ORIGINAL, x=None, noalloc=False):
        """b: float64 device tensor of shape (n,) or (nrhs, n) (column c = b[c]).
        noalloc=True calls sptrsv_solve_noalloc (work vectors in the library's
        static work area; x must be given and the schedule prepared)."""
        _need(b.dtype == torch.float64 and b.is_cuda, "float64 device tensor expected")
        bb = b if b.dim() == 2 else b.view(1, -1)
        _need(bb.shape[1] == self.n and bb.stride(1) == 1, "b must be (nrhs, n) with unit row stride")
        nrhs = bb.shape[0]
        ldb = bb.stride(0) if nrhs > 1 else self.n
        if x is None:
            x = torch.empty_like(bb)
        xx = x if x.dim() == 2 else x.view(1, -1)
        ldx = xx.stride(0) if nrhs > 1 else self.n
        fn = self._L.sptrsv_solve_noalloc if noalloc else self._L.sptrsv_solve
        self._check(fn(self._h, which, nrhs, _ptr(bb), ldb, _ptr(xx), ldx, _stream()))
        return x if b.dim() == 2 else x.view(-1)

    def solve_rows(self, b, which=ORIGINAL, x=None):
        """b: float64 device tensor of shape (n, nrhs), contiguous (a row's
        right-hand sides together); returns x of the same shape."""
        _need(b.dtype == torch.float64 and b.is_cuda and b.dim() == 2 and b.shape[0] == self.n and b.is_contiguous(),
              "contiguous float64 device tensor of shape (n, nrhs) expected")
        if x is None:
            x = torch.empty_like(b)
        _need(x.shape == b.shape and x.is_contiguous(), "x must be a contiguous (n, nrhs) tensor")
        self._check(self._L.sptrsv_solve_rows(self._h, which, b.shape[1], _ptr(b), _ptr(x), _stream()))
        return x

    def graph_create_rows(self, b, x, which=ORIGINAL) -> int:
        _need(b.is_contiguous() and x.is_contiguous() and b.shape == x.shape and b.dim() == 2, "(n, nrhs) tensors")
        gid = C.c_int32(0)
        self._check(self._L.sptrsv_graph_create_rows(self._h, which, b.shape[1], _ptr(b), _ptr(x), _stream(),
                                                     C.byref(gid)))
        self._keep.append((b, x))
        return gid.value

    def prepare(self, which=ORIGINAL, nrhs=1):
        self._check(self._L.sptrsv_prepare(self._h, which, nrhs, _stream()))

    def check(self):
        self._check(self._L.sptrsv_check(self._h, _stream()))

    def residual(self, b, x):
        bb = b if b.dim() == 2 else b.view(1, -1)
        xx = x if x.dim() == 2 else x.view(1, -1)
        nrhs = bb.shape[0]
        out = (C.c_double * nrhs)()
        self._check(self._L.sptrsv_residual(self._h, nrhs, _ptr(bb), bb.stride(0) if nrhs > 1 else self.n,
                                            _ptr(xx), xx.stride(0) if nrhs > 1 else self.n, out, _stream()))
        return list(out)

    def set_schedule(self, which=ORIGINAL, mode=0, thin_rows=4096, wg_threads=512, wide_threads=256,
                     lanes_per_row=1, wide_grid=0, overlap=0, thin_cols=0):
        s = Schedule(mode, thin_rows, wg_threads, wide_threads, lanes_per_row, wide_grid, overlap, thin_cols)
        self._check(self._L.sptrsv_set_schedule(self._h, which, C.byref(s)))

    def get_schedule(self, which=ORIGINAL, nrhs=1):
        """The schedule a solve with nrhs right-hand sides uses."""
        s = Schedule()
        self._check(self._L.sptrsv_get_schedule(self._h, which, nrhs, C.byref(s)))
        return s.as_dict()

    def autotune(self, which=ORIGINAL, nrhs=1, rows=False) -> float:
        """Tunes the schedule of (which, nrhs); rows: timing solves with the
        right-hand sides stored by rows. Returns the best time in ms."""
        ms = C.c_float(0)
        fn = self._L.sptrsv_autotune_rows if rows else self._L.sptrsv_autotune
        self._check(fn(self._h, which, nrhs, _stream(), C.byref(ms)))
        return ms.value

    def measure_level_costs(self) -> dict:
        """ns per empty level for each way a solve separates levels."""
        out = LevelCosts()
        self._check(self._L.sptrsv_measure_level_costs(self._h, _stream(), C.byref(out)))
        return out.as_dict()

    def level_floor(self, costs: dict, which=ORIGINAL, nrhs=1, graph=False, rows=False) -> float:
        """Microseconds one solve of (which, nrhs) costs at least with empty
        levels, under the schedule it uses (rows: right-hand sides by rows)."""
        c = LevelCosts(**costs)
        out = C.c_double(0)
        flags = (1 if graph else 0) | (2 if rows else 0)
        self._check(self._L.sptrsv_level_floor(self._h, which, nrhs, flags, C.byref(c), C.byref(out)))
        return out.value

    def tune_info(self) -> dict:
        """What the last autotune did: candidates timed, candidates dropped at
        their device-side wait limit, the best time and the largest limit."""
        out = TuneInfo()
        self._check(self._L.sptrsv_get_tune_info(self._h, C.byref(out)))
        return out.as_dict()

    def profile_start(self):
        self._check(self._L.sptrsv_profile(self._h, 1, None, _stream()))

    def profile_stop(self):
        out = (KernelProfile * 4)()
        self._check(self._L.sptrsv_profile(self._h, 0, out, _stream()))
        return {PROFILE_CLASSES[i]: dict(launches=out[i].launches, ms=out[i].ms, bytes=out[i].bytes)
                for i in range(4)}

    def graph_create(self, b, x, which=ORIGINAL) -> int:
        bb = b if b.dim() == 2 else b.view(1, -1)
        xx = x if x.dim() == 2 else x.view(1, -1)
        nrhs = bb.shape[0]
        gid = C.c_int32(0)
        self._check(self._L.sptrsv_graph_create(self._h, which, nrhs, _ptr(bb), bb.stride(0) if nrhs > 1 else self.n,
                                                _ptr(xx), xx.stride(0) if nrhs > 1 else self.n, _stream(),
                                                C.byref(gid)))
        self._keep.append((b, x))
        return gid.value

    def graph_launch(self, gid: int):
        self._check(self._L.sptrsv_graph_launch(self._h, gid, _stream()))

    # ------------------------------------------------------------------- batched
    def batch_analyze(self, ns, row_ptr_cat, col_cat, val_cat):
        """ns: list of sizes; *_cat: concatenated device arrays (local indices;
        row pointers of matrix i occupy n_i+1 entries)."""
        import numpy as np
        ns = np.asarray(ns, np.int32)
        row_off = np.zeros(len(ns), np.int64)
        row_off[1:] = np.cumsum(ns.astype(np.int64))[:-1]
        self._bn = ns
        self._brow_off = row_off
        nnz_off = np.zeros(len(ns), np.int64)
        rp_host = row_ptr_cat.cpu().numpy()
        acc = 0
        for i in range(len(ns)):
            nnz_off[i] = acc
            acc += int(rp_host[row_off[i] + i + ns[i]])
        self._check(self._L.sptrsv_batch_analyze(self._h, len(ns), ns.ctypes.data, row_off.ctypes.data,
                                                 nnz_off.ctypes.data, _ptr(row_ptr_cat), _ptr(col_cat),
                                                 _ptr(val_cat), _stream()))
        return nnz_off

    def batch_solve(self, b_cat, x_cat, nrhs: int, looped: bool = False):
        f = self._L.sptrsv_batch_solve_looped if looped else self._L.sptrsv_batch_solve
        self._check(f(self._h, nrhs, _ptr(b_cat), _ptr(x_cat), _stream()))
        return x_cat

    def batch_levels(self, i: int):
        nl = C.c_int32(0)
        self._check(self._L.sptrsv_batch_levels(self._h, i, C.byref(nl), None, None, _stream()))
        n = int(self._bn[i])
        lp = torch.empty(nl.value + 1, dtype=torch.int32, device="cuda")
        lr = torch.empty(n, dtype=torch.int32, device="cuda")
        self._check(self._L.sptrsv_batch_levels(self._h, i, C.byref(nl), _ptr(lp), _ptr(lr), _stream()))
        return lp, lr

    # ---------------------------------------------------------------- plan files
    def plan_save(self, path: str):
        self._check(self._L.sptrsv_plan_save(self._h, path.encode()))

    def plan_load(self, path: str):
        """Replace this handle's analysis and rewrite by a plan file's."""
        self._check(self._L.sptrsv_plan_load(self._h, path.encode()))
        info, st = Info(), RewriteStats()
        self._check(self._L.sptrsv_get_info(self._h, C.byref(info), C.byref(st)))
        self.n, self.nlev = info.n, info.nlev
        self.rstats = st.as_dict() if info.has_rewrite else None
        return {"form": info.form, "n": info.n, "nnz": info.nnz, "nlev": info.nlev,
                "has_rewrite": bool(info.has_rewrite)}

    # ------------------------------------------------------------ learned policy
    def level_times(self, b, which=ORIGINAL):
        """Per-level device time (ns) of one solve with every level in one workgroup."""
        bb = b if b.dim() == 2 else b.view(1, -1)
        nlev = self.nlev if which == ORIGINAL else self.rstats["nlev_after"]
        t = torch.empty(nlev, dtype=torch.float32, device="cuda")
        self._check(self._L.sptrsv_level_times(self._h, which, bb.shape[0], _ptr(bb.contiguous()), _ptr(t), _stream()))
        return t

    def level_finish_times(self, b, which=ORIGINAL):
        """Per-level finish times (ns from the solve's first written value) of
        one synchronisation-free solve."""
        bb = b if b.dim() == 2 else b.view(1, -1)
        nlev = self.nlev if which == ORIGINAL else self.rstats["nlev_after"]
        t = torch.empty(nlev, dtype=torch.float32, device="cuda")
        self._check(self._L.sptrsv_level_finish_times(self._h, which, bb.shape[0], _ptr(bb.contiguous()), _ptr(t),
                                                      _stream()))
        return t

    def level_features(self):
        f = torch.empty((self.nlev, MLP_NIN), dtype=torch.float32, device="cuda")
        self._check(self._L.sptrsv_level_features(self._h, _ptr(f), _stream()))
        return f
