"""Pins for the oracle's validation, forward substitution, level sets and
cost model, each against something other than the oracle itself: closed forms,
library routines, error bounds, brute force and the paper's worked examples."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import gen
import oracle


# ----------------------------------------------------------------- O1 validate
def _csr(n, rows):
    rp, ci, v = [0], [], []
    for r in rows:
        for c, x in r:
            ci.append(c)
            v.append(x)
        rp.append(len(ci))
    return gen.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64), "t")


@pytest.mark.parametrize("rows,expect", [
    ([[(0, 2.0)], [(0, 1.0), (1, 3.0)]], "OK"),
    ([[(0, 2.0)], [(1, 3.0), (0, 1.0)]], "UNSORTED"),          # descending columns
    ([[(0, 2.0)], [(0, 1.0), (0, 1.0), (1, 3.0)]], "UNSORTED"),  # duplicate column
    ([[(0, 2.0), (1, 1.0)], [(1, 3.0)]], "NOT_LOWER"),          # upper-triangle entry
    ([[(0, 2.0)], [(0, 1.0)]], "MISSING_DIAG"),                 # no diagonal
    ([[(0, 2.0)], []], "MISSING_DIAG"),                         # empty row
    ([[(0, 0.0)], [(0, 1.0), (1, 3.0)]], "ZERO_PIVOT"),
    ([[(0, 2.0)], [(0, np.nan), (1, 3.0)]], "NONFINITE"),
    ([[(0, np.inf)], [(0, 1.0), (1, 3.0)]], "NONFINITE"),
    ([[(0, 2.0)], [(1, 3.0), (0, 1.0)], [(3, 1.0), (2, 1.0)]], "NOT_LOWER"),  # priority
])
def test_validate_cases(rows, expect):
    assert oracle.validate(_csr(len(rows), rows)) == expect


def test_validate_bad_row_ptr():
    m = gen.window_random(50, 1)
    rp = m.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]
    assert oracle.validate(gen.Csr(m.n, rp, m.col, m.val)) == "ARG"


def test_generated_inputs_valid_and_dominant():
    for m in [gen.window_random(500, 3), gen.stencil2d_chain(12, 40, 1), gen.stencil3d_tail(5, 20, 4),
              gen.powerlaw(3000, 5, w_loc=64, nseg=2, seglen=30)]:
        assert oracle.validate(m) == "OK"
        d = m.val[m.row_ptr[1:] - 1]
        off = np.add.reduceat(np.abs(m.val), m.row_ptr[:-1]) - np.abs(d)
        assert np.all(d >= 1.0 + off - 1e-12)


# ------------------------------------------------------------- O2 forward subst
def test_diagonal_is_one_division():
    m = gen.diagonal(300, 7)
    b = gen.rhs(m, 3)
    x = oracle.solve(m, b)
    assert np.array_equal(x, b / m.val[None, :])  # exactly one rounding per entry


def test_constant_bidiagonal_closed_form():
    # L = d I + e S (S = subdiagonal shift): x_i = sum_{k<=i} (-e/d)^{i-k} b_k / d
    n, d, e = 40, 2.5, -1.25
    rows = [[(0, d)]] + [[(i - 1, e), (i, d)] for i in range(1, n)]
    m = _csr(n, rows)
    rng = np.random.default_rng(0)
    b = rng.uniform(-1, 1, (2, n))
    x = oracle.solve(m, b)
    i = np.arange(n)
    P = np.where(i[:, None] >= i[None, :], (-e / d) ** (i[:, None] - i[None, :]).clip(0), 0.0) / d
    xref = b @ P.T
    assert oracle.relerr(x, xref) < 1e-14


def test_ones_vector_from_L_times_ones():
    m = gen.window_random(2000, 0)
    b = (m.to_scipy() @ np.ones(m.n))[None, :]
    x = oracle.solve(m, b)
    assert np.max(np.abs(x - 1.0)) < 1e-13


def test_dense_against_lapack():
    rng = np.random.default_rng(5)
    n = 200
    a = np.tril(rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.1), -1)
    a[np.diag_indices(n)] = 1.0 + np.abs(a).sum(1)
    m = gen.from_dense_lower(a)
    b = rng.uniform(-1, 1, (4, n))
    x = oracle.solve(m, b)
    xr = sla.solve_triangular(a, b.T, lower=True).T
    assert oracle.relerr(x, xr) < 1e-13


def test_config0_against_scipy_sparse():
    m, _ = gen.config_matrix(0)
    b = gen.rhs(m, 1)
    x = oracle.solve(m, b)
    xr = spla.spsolve_triangular(m.to_scipy().tocsr(), b[0], lower=True)
    assert oracle.relerr(x, xr[None]) < 1e-13


def test_residual_backward_stable_and_varah():
    # backward stability of substitution: |b - L x| <= gamma_k |L| |x|; Varah:
    # ||L^{-1}||_inf <= 1 / min_i (|l_ii| - sum_j |l_ij|) = 1 for these inputs.
    m = gen.stencil2d_chain(30, 200, 1)
    b = gen.rhs(m, 2)
    x = oracle.solve(m, b)
    A = m.to_scipy()
    absA = abs(A)
    kmax = int(np.max(np.diff(m.row_ptr)))
    gam = kmax * np.finfo(float).eps / (1 - kmax * np.finfo(float).eps)
    for c in range(2):
        r = np.abs(b[c] - A @ x[c])
        assert np.all(r <= 1.01 * gam * (absA @ np.abs(x[c])) + 1e-300)
        assert np.max(np.abs(x[c])) <= np.max(np.abs(b[c])) * (1 + 1e-12)


# -------------------------------------------------------------------- O3 levels
def _bf_levels(m):
    """Longest path by memoised depth-first search (pure Python)."""
    import sys
    sys.setrecursionlimit(100000)
    memo = {}

    def lev(r):
        if r in memo:
            return memo[r]
        deps = m.col[m.row_ptr[r]:m.row_ptr[r + 1] - 1]
        v = 0 if len(deps) == 0 else 1 + max(lev(int(j)) for j in deps)
        memo[r] = v
        return v

    return np.array([lev(r) for r in range(m.n)], np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_levels_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    m = gen.window_random(n, seed, window=int(rng.integers(1, 20)), draws=int(rng.integers(1, 6)))
    lv = oracle.levels(m)
    bf = _bf_levels(m)
    assert np.array_equal(lv.row_level, bf)
    assert lv.nlev == (bf.max() + 1 if n else 0)
    order = np.lexsort((np.arange(n), bf))
    assert np.array_equal(lv.level_rows, order)
    assert np.array_equal(lv.level_ptr, np.concatenate([[0], np.cumsum(np.bincount(bf))]))


def test_levels_closed_forms():
    assert oracle.levels(gen.diagonal(50)).nlev == 1
    lv = oracle.levels(gen.bidiagonal(77))
    assert lv.nlev == 77 and np.array_equal(lv.row_level, np.arange(77))
    k, chain = 20, 30
    lv = oracle.levels(gen.stencil2d_chain(k, chain, 1))
    p = np.arange(k * k)
    assert np.array_equal(lv.row_level[:k * k], p // k + p % k)
    assert lv.nlev == 2 * k - 1 + chain
    w = np.diff(lv.level_ptr)[:2 * k - 1]
    ell = np.arange(2 * k - 1)
    assert np.array_equal(w, np.minimum(ell + 1, 2 * k - 1 - ell))
    k3 = 7
    lv = oracle.levels(gen.stencil3d_tail(k3, 15, 4))
    p = np.arange(k3 ** 3)
    assert np.array_equal(lv.row_level[:k3 ** 3], p // (k3 * k3) + (p // k3) % k3 + p % k3)
    assert lv.nlev == 3 * k3 - 2 + 15


def test_config1_level_count():
    lv = oracle.levels(gen.stencil2d_chain(1000, 20000, 1))
    assert lv.nlev == 21999


def test_level_invariants_powerlaw():
    m = gen.powerlaw(20000, 3, w_loc=128, nseg=3, seglen=40)
    lv = oracle.levels(m)
    lev = lv.row_level
    r = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    off = m.col != r
    # no dependency inside a level; every dependency is strictly earlier
    assert np.all(lev[m.col[off]] < lev[r[off]])
    # every row above level 0 has a dependency exactly one level up
    best = np.full(m.n, -1)
    np.maximum.at(best, r[off], lev[m.col[off]])
    assert np.all((lev == 0) | (best == lev - 1))


# ---------------------------------------------------------------- O4 cost model
def test_row7_example_cost():
    # Sec. II.A: row 7 reads rows 0, 3 and 6; cost of a row = 2*nnz - 1 (Sec. III)
    with open(os.path.join(os.path.dirname(__file__), "golden", "row7_example.json")) as f:
        g = json.load(f)
    r7 = g["row"]
    rows = [[(i, 2.0)] for i in range(r7)] + [[(d, .1 * (k + 1)) for k, d in enumerate(g["dependencies"])] + [(r7, 2.0)]]
    rows[3] = [(1, .5), (3, 2.0)]
    rows[6] = [(3, .5), (6, 2.0)]
    m = _csr(r7 + 1, rows)
    assert m.row_ptr[r7 + 1] - m.row_ptr[r7] == g["nnz"]
    lv = oracle.levels(m)
    assert lv.row_level[r7] == 1 + max(lv.row_level[g["dependencies"]])
    c = oracle.level_costs(m, lv)
    assert c.cost[lv.row_level[r7]] == g["cost"]  # the only row of its level


def fig2_matrix(v00=2.0, v10=0.5, v11=3.0, v22=1.5, v31=-0.75, v33=4.0):
    """Fig. 2: row 3 reads row 1, which reads row 0; row 2 is independent."""
    return _csr(4, [[(0, v00)], [(0, v10), (1, v11)], [(2, v22)], [(1, v31), (3, v33)]])


def test_fig2_costs_before():
    m = fig2_matrix()
    nnz = np.diff(m.row_ptr)
    assert 2 * nnz[1] - 1 == 3 and 2 * nnz[3] - 1 == 3  # Sec. III: rows 1 and 3 cost 3
    lv = oracle.levels(m)
    c = oracle.level_costs(m, lv)
    assert c.total == int(np.sum(2 * nnz - 1))
    assert c.avg == c.total / lv.nlev


# ---------------------------------------- upper-triangular and transposed forms
def _upper_of(m):
    return oracle.transpose(m)


def test_upper_bidiagonal_closed_form():
    # U = 2 on the diagonal, -1 above it; b = U 1 gives x = 1 exactly
    n = 57
    rp = np.arange(0, 2 * n, 2, dtype=np.int32)
    rp = np.append(rp, 2 * n - 1).astype(np.int32)
    ci = np.empty(2 * n - 1, np.int32)
    va = np.empty(2 * n - 1)
    for i in range(n):
        ci[2 * i] = i
        va[2 * i] = 2.0
        if i + 1 < n:
            ci[2 * i + 1] = i + 1
            va[2 * i + 1] = -1.0
    u = gen.Csr(n, rp, ci, va, "upper_bidiag")
    b = np.ones((1, n))
    b[0, -1] = 2.0
    assert np.array_equal(oracle.solve_upper(u, b), np.ones((1, n)))


@pytest.mark.parametrize("seed", range(4))
def test_upper_and_transposed_forms_against_dense(seed):
    import scipy.linalg as sla
    m = gen.window_random(150 + 7 * seed, seed, window=9, draws=3)
    u = _upper_of(gen.window_random(150 + 7 * seed, 50 + seed, window=9, draws=3))
    b = gen.rhs(m, 3)
    L, U = m.to_scipy().toarray(), u.to_scipy().toarray()
    for form, mat, dense in ((oracle.UPPER, u, U), (oracle.LOWER_TRANS, m, L.T), (oracle.UPPER_TRANS, u, U.T),
                             (oracle.LOWER, m, L)):
        x = oracle.solve_form(mat, b, form)
        xr = sla.solve_triangular(dense, b.T, lower=form in (oracle.LOWER, oracle.UPPER_TRANS)).T
        assert oracle.relerr(x, xr) < 1e-12, form
        # and the residual of the system itself
        assert np.abs(dense @ x.T - b.T).max() <= 1e-12 * (1.0 + np.abs(b).max())


def test_reversal_turns_upper_into_lower():
    # J U J (rows and columns in reverse order) is lower-triangular with the
    # diagonal last, and solving it on J b gives J x
    u = _upper_of(gen.window_random(300, 4, window=20, draws=4))
    n = u.n
    nnz = u.nnz
    rp = (nnz - u.row_ptr[::-1]).astype(np.int32)
    ci = (n - 1 - u.col[::-1]).astype(np.int32)
    va = u.val[::-1].copy()
    r = gen.Csr(n, rp, ci, va, "JUJ")
    assert oracle.validate(r) == "OK"
    b = gen.rhs(u, 2)
    x = oracle.solve_upper(u, b)
    xr = oracle.solve(r, b[:, ::-1].copy())[:, ::-1]
    assert oracle.relerr(xr, x) < 1e-13
