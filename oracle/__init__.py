"""CPU oracle for rewritten level-set SpTRSV (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. It shares no code with the HIP library and never
calls it. The arithmetic lives in ``oracle.c`` (serial, FP64, compiled without
FMA contraction); this module loads it with ctypes and adds the FP64 MLP oracle
(``mlp.py``).

Functions and the paper passages they follow (arXiv 2206.05843):
  validate        CSR well-formedness, diagonal last        Sec. II.A, Algorithm 1
  solve           serial forward substitution               Sec. II.A, Algorithm 1
  levels          level sets by longest dependency path     Sec. II.A
  level_costs     2*nnz-1 per row, avgLevelCost             Sec. III, cost model
  rewrite         thin/target/source scan + substitution    Sec. II.B, Sec. III; row constraints
                  Sec. III.A; both_ends: segments taken from both ends (Sec. III, parallel sketch)
  spmv            b' = T b                                  Sec. II.B (rearrangement)
  solve_upper / solve_form  U x = b and transposed forms    Sec. I (preconditioner use)
  level_features  learned-policy inputs                     no paper passage for 0..15; 16..19 are the
                  Sec. III.A row constraints measured per level (see oracle.c)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "OK", 1: "ARG", 2: "NOT_LOWER", 3: "UNSORTED", 4: "MISSING_DIAG", 5: "ZERO_PIVOT",
          6: "NONFINITE", 7: "ALLOC", 8: "OVERFLOW"}

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
                               "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB_PATH)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    lib.orc_validate.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p]
    lib.orc_validate.restype = C.c_int
    lib.orc_solve.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, f64p, C.c_int64, f64p, C.c_int64]
    lib.orc_solve.restype = None
    lib.orc_spmv.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, f64p, C.c_int64, f64p, C.c_int64]
    lib.orc_spmv.restype = None
    lib.orc_levels.argtypes = [C.c_int32, i32p, i32p, i32p, i32p, i32p]
    lib.orc_levels.restype = C.c_int32
    lib.orc_level_costs.argtypes = [C.c_int32, i32p, C.c_int32, i32p, i32p, i64p, i64p, i64p,
                                    C.POINTER(C.c_int64)]
    lib.orc_level_costs.restype = C.c_double
    lib.orc_solve_upper.argtypes = lib.orc_solve.argtypes
    lib.orc_solve_upper.restype = None
    lib.orc_rewrite.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p, i32p, C.c_int32,
                                C.c_double, C.c_double, C.c_int32, C.c_void_p, i32p, C.POINTER(C.c_int32)]
    lib.orc_rewrite.restype = C.c_void_p
    lib.orc_rewrite_rc.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p, i32p, C.c_int32,
                                   C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                   C.c_int32, i32p, C.POINTER(C.c_int32)]
    lib.orc_rewrite_rc.restype = C.c_void_p
    lib.orc_rewrite_lv.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p, i32p, C.c_int32,
                                   C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                   C.c_int32, C.c_void_p, C.c_void_p, i32p, C.POINTER(C.c_int32)]
    lib.orc_rewrite_lv.restype = C.c_void_p
    lib.orc_rewrite_skipped.argtypes = [C.c_void_p]
    lib.orc_rewrite_skipped.restype = C.c_int32
    lib.orc_rewrite_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.orc_rewrite_sizes.restype = None
    lib.orc_rewrite_copy.argtypes = [C.c_void_p, i32p, i32p, f64p, i32p, i32p, f64p]
    lib.orc_rewrite_copy.restype = None
    lib.orc_rewrite_free.argtypes = [C.c_void_p]
    lib.orc_rewrite_free.restype = None
    lib.orc_level_features.argtypes = [C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p, i32p, f64p]
    lib.orc_level_features.restype = C.c_int
    _lib = lib
    return lib


def _arrs(m):
    return (np.ascontiguousarray(m.row_ptr, np.int32), np.ascontiguousarray(m.col, np.int32),
            np.ascontiguousarray(m.val, np.float64))


def validate(m) -> str:
    rp, ci, v = _arrs(m)
    return STATUS[_load().orc_validate(m.n, int(rp[-1]) if rp.size else 0, rp, ci, v)]


def solve(m, b: np.ndarray) -> np.ndarray:
    """x = L^{-1} b by Algorithm 1. ``b`` has shape (nrhs, n) (column-major)."""
    rp, ci, v = _arrs(m)
    b = np.ascontiguousarray(np.atleast_2d(b), np.float64)
    x = np.zeros_like(b)
    _load().orc_solve(m.n, rp, ci, v, b.shape[0], b, m.n, x, m.n)
    return x


def solve_upper(m, b: np.ndarray) -> np.ndarray:
    """x = U^{-1} b by backward substitution; ``m`` upper-triangular CSR with
    the diagonal first in each row; ``b`` has shape (nrhs, n)."""
    rp, ci, v = _arrs(m)
    b = np.ascontiguousarray(np.atleast_2d(b), np.float64)
    x = np.zeros_like(b)
    _load().orc_solve_upper(m.n, rp, ci, v, b.shape[0], b, m.n, x, m.n)
    return x


def transpose(m):
    """The transpose as a CSR with sorted rows (a plain library transpose)."""
    import scipy.sparse as sps
    from gen import Csr
    a = sps.csr_matrix((m.val, m.col, m.row_ptr), shape=(m.n, m.n)).T.tocsr()
    a.sort_indices()
    return Csr(m.n, a.indptr.astype(np.int32), a.indices.astype(np.int32), a.data.astype(np.float64), m.name + "^T")


LOWER, UPPER, LOWER_TRANS, UPPER_TRANS = 0, 1, 2, 3


def solve_form(m, b: np.ndarray, form: int) -> np.ndarray:
    """x for the system ``m`` stands for: L x = b (LOWER), U x = b (UPPER),
    L^T x = b (LOWER_TRANS, m lower) or U^T x = b (UPPER_TRANS, m upper)."""
    if form == LOWER:
        return solve(m, b)
    if form == UPPER:
        return solve_upper(m, b)
    if form == LOWER_TRANS:
        return solve_upper(transpose(m), b)
    if form == UPPER_TRANS:
        return solve(transpose(m), b)
    raise ValueError(form)


def spmv(rp, ci, v, n, b: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(np.atleast_2d(b), np.float64)
    y = np.zeros_like(b)
    _load().orc_spmv(n, np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
                     np.ascontiguousarray(v, np.float64), b.shape[0], b, n, y, n)
    return y


@dataclass
class Levels:
    nlev: int
    row_level: np.ndarray   # int32[n]
    level_ptr: np.ndarray   # int32[nlev+1]
    level_rows: np.ndarray  # int32[n]


def levels(m) -> Levels:
    rp, ci, _ = _arrs(m)
    lev = np.zeros(m.n, np.int32)
    lptr = np.zeros(m.n + 1, np.int32)
    lrows = np.zeros(m.n, np.int32)
    nlev = _load().orc_levels(m.n, rp, ci, lev, lptr, lrows)
    return Levels(int(nlev), lev, lptr[:nlev + 1].copy(), lrows)


@dataclass
class Costs:
    rows: np.ndarray
    nnz: np.ndarray
    cost: np.ndarray
    total: int
    avg: float


def level_costs(m, lv: Levels | None = None) -> Costs:
    lv = lv or levels(m)
    rp, _, _ = _arrs(m)
    rows = np.zeros(lv.nlev, np.int64)
    nz = np.zeros(lv.nlev, np.int64)
    cost = np.zeros(lv.nlev, np.int64)
    tot = C.c_int64(0)
    avg = _load().orc_level_costs(m.n, rp, lv.nlev, lv.level_ptr, lv.level_rows, rows, nz, cost, C.byref(tot))
    return Costs(rows, nz, cost, int(tot.value), float(avg))


@dataclass
class Rewrite:
    n: int
    lp_ptr: np.ndarray
    lp_col: np.ndarray
    lp_val: np.ndarray
    t_ptr: np.ndarray
    t_col: np.ndarray
    t_val: np.ndarray
    target: np.ndarray      # int32[n], -1 = row not rewritten
    rows_rewritten: int
    max_distance: int
    steps: int
    rows_skipped: int = 0   # rows a row constraint left in place

    @property
    def lp(self):
        from gen import Csr
        return Csr(self.n, self.lp_ptr, self.lp_col, self.lp_val, "L'")

    @property
    def t(self):
        from gen import Csr
        return Csr(self.n, self.t_ptr, self.t_col, self.t_val, "T")


THIN_ROWS, THIN_COST = 0, 1
NFEAT = 20  # per-level features of the learned policy (see orc_level_features)


def rewrite(m, thin_metric: int = THIN_ROWS, thin_threshold: float = 32.0, fill_cap: float = 0.0,
            max_distance: int = 0, mask: np.ndarray | None = None, lv: Levels | None = None, max_indegree: int = 0,
            max_spread: int = 0, critical_only: bool = False, both_ends: bool = False,
            level_budget: np.ndarray | None = None, level_cap: np.ndarray | None = None) -> Rewrite:
    """The scan and rewriting of Sec. II.B / Sec. III (oracle.c O5), with the
    row constraints of Sec. III.A: max_indegree (alpha), max_spread (beta) and
    critical_only; 0 / False disable them. both_ends takes the independent
    segments of the scan alternately from the first and the last level (the
    result is the same). level_budget (int32 per level, rows, THIN_ROWS) and
    level_cap (float32 per level) replace thin_threshold and fill_cap for the
    rows of a source level where they are positive."""
    lib = _load()
    lv = lv or levels(m)
    rp, ci, v = _arrs(m)
    tgt = np.zeros(m.n, np.int32)
    st = C.c_int32(0)
    mk = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, np.uint8)
        assert mk.size >= lv.nlev
    lb = lc = None
    if level_budget is not None:
        lb = np.ascontiguousarray(level_budget, np.int32)
        assert lb.size >= lv.nlev
    if level_cap is not None:
        lc = np.ascontiguousarray(level_cap, np.float32)
        assert lc.size >= lv.nlev
    ctx = lib.orc_rewrite_lv(m.n, rp, ci, v, lv.nlev, lv.row_level, lv.level_ptr, lv.level_rows, thin_metric,
                             float(thin_threshold), float(fill_cap), int(max_distance),
                             mk.ctypes.data if mk is not None else None, int(max_indegree), int(max_spread),
                             int(bool(critical_only)), int(bool(both_ends)),
                             lb.ctypes.data if lb is not None else None, lc.ctypes.data if lc is not None else None,
                             tgt, C.byref(st))
    if not ctx:
        raise RuntimeError(f"oracle rewrite failed: {STATUS[st.value]}")
    try:
        a, b = C.c_int64(0), C.c_int64(0)
        rr, md, steps = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        lib.orc_rewrite_sizes(ctx, C.byref(a), C.byref(b), C.byref(rr), C.byref(md), C.byref(steps))
        lp_ptr = np.zeros(m.n + 1, np.int32)
        t_ptr = np.zeros(m.n + 1, np.int32)
        lp_col = np.zeros(a.value, np.int32)
        lp_val = np.zeros(a.value, np.float64)
        t_col = np.zeros(b.value, np.int32)
        t_val = np.zeros(b.value, np.float64)
        lib.orc_rewrite_copy(ctx, lp_ptr, lp_col, lp_val, t_ptr, t_col, t_val)
        skipped = lib.orc_rewrite_skipped(ctx)
    finally:
        lib.orc_rewrite_free(ctx)
    return Rewrite(m.n, lp_ptr, lp_col, lp_val, t_ptr, t_col, t_val, tgt, rr.value, md.value, steps.value, skipped)


def rewrite_stats(m, rw: Rewrite, lv: Levels | None = None) -> dict:
    """Table I style metrics (Sec. IV): levels, total and average level cost,
    rows rewritten, before and after, plus nnz of L, L' and T."""
    lv = lv or levels(m)
    cb = level_costs(m, lv)
    lv2 = levels(rw.lp)
    ca = level_costs(rw.lp, lv2)
    return dict(nlev_before=lv.nlev, nlev_after=lv2.nlev, rows_rewritten=rw.rows_rewritten,
                max_distance=rw.max_distance, nnz_L=m.nnz, nnz_Lp=int(rw.lp_ptr[-1]), nnz_T=int(rw.t_ptr[-1]),
                total_cost_before=cb.total, total_cost_after=ca.total, avg_level_cost_before=cb.avg,
                avg_level_cost_after=ca.avg)


def solve_rewritten(rw: Rewrite, b: np.ndarray) -> np.ndarray:
    """x from the rewritten system: b' = T b, then Algorithm 1 on (L', b')."""
    bp = spmv(rw.t_ptr, rw.t_col, rw.t_val, rw.n, b)
    return solve(rw.lp, bp)


def level_features(m, lv: Levels | None = None) -> np.ndarray:
    lv = lv or levels(m)
    rp, ci, v = _arrs(m)
    f = np.zeros((lv.nlev, NFEAT), np.float64)
    st = _load().orc_level_features(m.n, rp, ci, v, lv.nlev, lv.row_level, lv.level_ptr, lv.level_rows, f)
    if st != 0:
        raise RuntimeError(STATUS[st])
    return f


def relerr(x: np.ndarray, xref: np.ndarray) -> float:
    """max over RHS columns of ||x_c - xref_c||_inf / ||xref_c||_inf."""
    x = np.atleast_2d(x)
    xref = np.atleast_2d(xref)
    num = np.max(np.abs(x - xref), axis=1)
    den = np.maximum(np.max(np.abs(xref), axis=1), np.finfo(np.float64).tiny)
    return float(np.max(num / den)) if x.size else 0.0
