"""Pins for the oracle's rewriting (substitution, rearrangement and the naive
strategy's scan): the paper's Fig. 2 closed form and its cost-map example, a
bidiagonal closed form, the unique-row characterisation by a dense solve,
reachability by breadth-first search, and invariants on random inputs."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from tests.test_oracle_solve_levels import _csr, fig2_matrix

THIN_ROWS, THIN_COST = oracle.THIN_ROWS, oracle.THIN_COST


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _row(rw_ptr, rw_col, rw_val, r):
    s, e = rw_ptr[r], rw_ptr[r + 1]
    return list(zip(rw_col[s:e].tolist(), rw_val[s:e].tolist()))


# ------------------------------------------------------------- Fig. 2 example
def test_fig2_closed_form():
    v00, v10, v11, v22, v31, v33 = 2.0, 0.5, 3.0, 1.5, -0.75, 4.0
    g = golden("fig2_example.json")
    m = fig2_matrix(v00, v10, v11, v22, v31, v33)
    for r, deps in g["dependencies"].items():
        s, e = m.row_ptr[int(r)], m.row_ptr[int(r) + 1]
        assert m.col[s:e - 1].tolist() == deps
    lv = oracle.levels(m)
    assert [lv_ + 1 for lv_ in lv.row_level] == g["levels_1based"]
    assert lv.nlev == max(g["levels_1based"])
    # first rewrite of row 3 (Fig. 2, middle): one level up, dependency on row 0
    rw1 = oracle.rewrite(m, THIN_ROWS, 100, mask=np.array([0, 0, 1], np.uint8))
    assert rw1.target[3] + 1 == g["row3_after_first_rewrite"]["level_1based"]
    assert [c for c, _ in _row(rw1.lp_ptr, rw1.lp_col, rw1.lp_val, 3)][:-1] == \
        g["row3_after_first_rewrite"]["dependencies"]
    # rewrite every level toward level 0 (the two substitutions of Fig. 2)
    rw = oracle.rewrite(m, THIN_ROWS, 100, mask=np.array([0, 1, 1], np.uint8))
    assert list(rw.target) == [-1, 0, -1, 0]
    assert rw.target[3] + 1 == g["row3_after_second_rewrite"]["level_1based"]
    l3 = _row(rw.lp_ptr, rw.lp_col, rw.lp_val, 3)
    t3 = _row(rw.t_ptr, rw.t_col, rw.t_val, 3)
    assert l3 == [(3, v33)]  # rewritten row keeps only its diagonal
    assert [c for c, _ in t3] == [0, 1, 3]
    np.testing.assert_allclose([x for _, x in t3], [v31 * v10 / (v11 * v00), -v31 / v11, 1.0], rtol=1e-15)
    # the rewritten x[3] equals the nested expression of Sec. II.B
    b = np.array([[0.3, -0.7, 0.2, 1.1]])
    x = oracle.solve_rewritten(rw, b)
    x3 = (b[0, 3] - v31 * ((b[0, 1] - v10 * (b[0, 0] / v00)) / v11)) / v33
    assert abs(x[0, 3] - x3) <= 4e-16 * abs(x3)
    # cost after rearrangement: row 3 costs 1 (Sec. III)
    assert 2 * (rw.lp_ptr[4] - rw.lp_ptr[3]) - 1 == g["row3_after_second_rewrite"]["cost_rearranged"]
    assert [c for c, _ in l3][:-1] == g["row3_after_second_rewrite"]["dependencies"]
    assert oracle.levels(rw.lp).nlev == 1


# -------------------------------------------------- cost-map worked example
def costmap_matrix():
    """Sec. III example shape: ancestors A..E at level 0, then levels n..n+3
    holding rows r0..r7 (indices 5..12). Level n is kept as a target via the
    mask; the budget is 22 as in the example."""
    A, B, Cc, D, E = range(5)
    r = list(range(5, 13))
    rows = [[(i, 4.0)] for i in range(5)]
    rows += [[(A, .1), (r[0], 4.0)], [(B, .1), (r[1], 4.0)]]              # level n
    rows += [[(r[0], .2), (r[2], 4.0)], [(r[1], .2), (r[3], 4.0)]]        # level n+1
    rows += [[(r[2], .3), (r[4], 4.0)],                                    # level n+2
             [(Cc, .1), (D, .1), (E, .1), (r[3], .3), (r[5], 4.0)]]
    rows += [[(r[5], .4), (r[6], 4.0)], [(r[4], .4), (r[7], 4.0)]]        # level n+3
    return _csr(13, rows)


def test_costmap_movement_pattern():
    g = golden("costmap_example.json")
    m = costmap_matrix()
    lv = oracle.levels(m)
    assert lv.nlev == 5
    r = list(range(5, 13))                    # example row i is matrix row r[i]
    lvl = {"n": 1, "n+1": 2, "n+2": 3, "n+3": 4}  # level 0 holds the ancestors
    for name, rows in g["levels"].items():
        assert [int(lv.row_level[r[i]]) for i in rows] == [lvl[name]] * len(rows)
    mask = np.array([0, 0, 1, 1, 1], np.uint8)
    rw = oracle.rewrite(m, THIN_COST, float(g["budget"]), mask=mask, lv=lv)
    tg = rw.target
    for i, name in g["moved"].items():
        assert tg[r[int(i)]] == lvl[name]
    for i in g["not_moved"]:
        assert tg[r[i]] == -1
    assert rw.rows_rewritten == len(g["moved"])
    lv2 = oracle.levels(rw.lp)
    assert lv2.nlev == lv.nlev - g["levels_removed"]
    # the example's final levels, below the ancestors' level
    for k, rows in enumerate(g["final_levels"]):
        got = sorted(int(x) for x in lv2.level_rows[lv2.level_ptr[k + 1]:lv2.level_ptr[k + 2]])
        assert [r.index(x) for x in got] == rows


# --------------------------------------------------- bidiagonal closed form
def test_bidiagonal_closed_form_config1_rule():
    n, W = 100, 32
    m = gen.bidiagonal(n, 11)
    d = m.val[m.row_ptr[1:] - 1]
    e = np.zeros(n)
    e[1:] = m.val[m.row_ptr[1:-1]]
    rw = oracle.rewrite(m, THIN_ROWS, W, fill_cap=4.0)
    assert oracle.levels(rw.lp).nlev == -(-n // W)
    for r in range(n):
        g, k = divmod(r, W)
        if k == 0:
            assert rw.target[r] == -1
            continue
        assert rw.target[r] == W * g  # targets are original level numbers
        p = W * g - 1
        lrow = _row(rw.lp_ptr, rw.lp_col, rw.lp_val, r)
        if g == 0:
            assert lrow == [(r, d[r])]
        else:
            val = (-1) ** k * e[r] * np.prod([e[r - q] / d[r - q] for q in range(1, k + 1)])
            assert [c for c, _ in lrow] == [p, r]
            assert abs(lrow[0][1] - val) <= 1e-14 * abs(val) and lrow[1][1] == d[r]
        trow = _row(rw.t_ptr, rw.t_col, rw.t_val, r)
        qs = range(1, (k if g > 0 else r) + 1)
        assert [c for c, _ in trow] == sorted([r - q for q in qs]) + [r]
        for c, tv in trow[:-1]:
            q = r - c
            ref = (-1) ** q * np.prod([e[r - mm] / d[r - mm - 1] for mm in range(q)])
            assert abs(tv - ref) <= 1e-13 * abs(ref)
        assert trow[-1] == (r, 1.0)


# ------------------------------------------------ invariants + brute force
def _final_cur(lv, rw):
    cur = lv.row_level.copy()
    mv = rw.target >= 0
    cur[mv] = rw.target[mv]
    return cur


def _reach(m, r, inB):
    """Breadth-first search from row r through rows in B: the B rows reached,
    and the rows outside B adjacent to them (or to r)."""
    seenB, A = set(), set()
    stack = [int(c) for c in m.col[m.row_ptr[r]:m.row_ptr[r + 1] - 1]]
    while stack:
        k = stack.pop()
        if inB[k]:
            if k not in seenB:
                seenB.add(k)
                stack.extend(int(c) for c in m.col[m.row_ptr[k]:m.row_ptr[k + 1] - 1])
        else:
            A.add(k)
    return seenB, A


def check_rewrite_invariants(m, rw, lv, thin_metric, thr, fill_cap, max_distance, mask=None):
    n = m.n
    L = m.to_scipy()
    Lp = rw.lp.to_scipy()
    T = rw.t.to_scipy()
    # L' = T L exactly in structure (values to rounding), T unit lower triangular
    assert oracle.validate(rw.lp) == "OK"
    assert oracle.validate(rw.t) == "OK"
    assert np.all(rw.t_val[rw.t_ptr[1:] - 1] == 1.0)
    prod = (T @ L).tocsr()
    prod.sort_indices()
    diff = abs(prod - Lp)
    scale = abs(T) @ abs(L)
    assert diff.max() <= 1e-12 * max(1.0, scale.max())
    cur = _final_cur(lv, rw)
    moved = rw.target >= 0
    assert rw.rows_rewritten == int(moved.sum())
    for r in range(n):
        if not moved[r]:
            assert _row(rw.lp_ptr, rw.lp_col, rw.lp_val, r) == list(
                zip(m.col[m.row_ptr[r]:m.row_ptr[r + 1]].tolist(), m.val[m.row_ptr[r]:m.row_ptr[r + 1]].tolist()))
            assert _row(rw.t_ptr, rw.t_col, rw.t_val, r) == [(r, 1.0)]
            continue
        t = rw.target[r]
        assert t < lv.row_level[r]
        if max_distance:
            assert lv.row_level[r] - t <= max_distance
        inB = cur >= t
        seenB, A = _reach(m, r, inB)
        lcols = rw.lp_col[rw.lp_ptr[r]:rw.lp_ptr[r + 1] - 1].tolist()
        tcols = rw.t_col[rw.t_ptr[r]:rw.t_ptr[r + 1] - 1].tolist()
        assert lcols == sorted(A)          # pattern of L'[r] = reachable A columns
        assert tcols == sorted(seenB)      # pattern of T[r]   = reachable B rows
        if fill_cap > 0:
            assert len(lcols) + 1 <= fill_cap * (m.row_ptr[r + 1] - m.row_ptr[r])
        # Appendix-style unique row: c = L[r,B] L[B,B]^{-1}, T[r,B] = -c
        Bl = sorted(seenB)
        if Bl:
            LBB = L[Bl][:, Bl].toarray()
            lrB = L[r, Bl].toarray().ravel()
            c = np.linalg.solve(LBB.T, lrB)
            tv = rw.t_val[rw.t_ptr[r]:rw.t_ptr[r + 1] - 1]
            np.testing.assert_allclose(tv, -c, rtol=1e-10, atol=1e-13)
    # re-levelled L': valid, never deeper
    lv2 = oracle.levels(rw.lp)
    assert lv2.nlev <= lv.nlev
    # same x from the rewritten system
    b = gen.rhs(m, 2)
    assert oracle.relerr(oracle.solve_rewritten(rw, b), oracle.solve(m, b)) < 1e-10
    return lv2


def _scan_replay(m, lv, rw, thin_metric, thr, fill_cap, max_distance, mask):
    """Re-derive the decisions from the per-row outcomes: every accepted row
    respects the budget, and each run stops exactly at the first refusal."""
    c = oracle.level_costs(m, lv)
    W = thr if (thin_metric == THIN_ROWS or thr > 0) else c.avg
    nnz_lp = np.diff(rw.lp_ptr)
    nnz_l = np.diff(m.row_ptr)
    t, size, cost = 0, c.rows[0], c.cost[0]
    for l in range(1, lv.nlev):
        src = bool(mask[l]) if mask is not None else (
            c.rows[l] < W if thin_metric == THIN_ROWS else c.cost[l] < W)
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        if not src:
            assert np.all(rw.target[rows] == -1)
            t, size, cost = l, c.rows[l], c.cost[l]
            continue
        for i, r in enumerate(rows):
            if rw.target[r] == t:
                size += 1
                cost += 2 * nnz_lp[r] - 1
                assert (size <= W) if thin_metric == THIN_ROWS else (cost <= W)
            else:
                assert rw.target[r] == -1 and np.all(rw.target[rows[i:]] == -1)
                t = l
                size = len(rows) - i
                cost = int(np.sum(2 * nnz_l[rows[i:]] - 1))
                break


CASES = [
    (THIN_ROWS, 4, 0.0, 0),
    (THIN_ROWS, 3, 2.0, 0),
    (THIN_ROWS, 6, 4.0, 2),
    (THIN_COST, 0.0, 0.0, 0),
    (THIN_COST, 0.0, 3.0, 0),
    (THIN_COST, 40.0, 0.0, 3),
]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("case", CASES)
def test_invariants_small_random(seed, case):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    m = gen.window_random(n, seed, window=int(rng.integers(1, 8)), draws=int(rng.integers(1, 4)))
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, *case, lv=lv)
    check_rewrite_invariants(m, rw, lv, *case)
    _scan_replay(m, lv, rw, *case, None)


@pytest.mark.parametrize("seed", range(4))
def test_invariants_with_mask(seed):
    rng = np.random.default_rng(7 + seed)
    m = gen.window_random(60, 20 + seed, window=5, draws=2)
    lv = oracle.levels(m)
    mask = (rng.random(lv.nlev) < 0.6).astype(np.uint8)
    rw = oracle.rewrite(m, THIN_ROWS, 8, 4.0, 0, mask, lv)
    check_rewrite_invariants(m, rw, lv, THIN_ROWS, 8, 4.0, 0, mask)
    _scan_replay(m, lv, rw, THIN_ROWS, 8, 4.0, 0, mask)


@pytest.mark.parametrize("mk", [lambda: gen.stencil2d_chain(10, 60, 1), lambda: gen.stencil3d_tail(4, 30, 4),
                                lambda: gen.powerlaw(800, 9, w_loc=16, nseg=2, seglen=25)])
def test_invariants_structured(mk):
    m = mk()
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, THIN_ROWS, 32, 4.0, 0, None, lv)
    check_rewrite_invariants(m, rw, lv, THIN_ROWS, 32, 4.0, 0)
    _scan_replay(m, lv, rw, THIN_ROWS, 32, 4.0, 0, None)


def test_paper_policy_thin_cost_default_budget():
    m = gen.stencil2d_chain(12, 80, 1)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, THIN_COST, 0.0, 0.0, 0, None, lv)
    st = oracle.rewrite_stats(m, rw, lv)
    assert st["nlev_after"] < st["nlev_before"]
    # Table I relation: average level cost = total / number of levels
    assert st["avg_level_cost_after"] == st["total_cost_after"] / st["nlev_after"]
    check_rewrite_invariants(m, rw, lv, THIN_COST, 0.0, 0.0, 0)


def test_config1_naive_structure():
    m = gen.stencil2d_chain(1000, 20000, 1)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, THIN_ROWS, 32, 4.0, 0, None, lv)
    st = oracle.rewrite_stats(m, rw, lv)
    assert st["nlev_before"] == 21999
    assert st["nlev_after"] < 6000
    # rows of the wide middle of the stencil are never touched
    mid = lv.level_rows[lv.level_ptr[900]:lv.level_ptr[1100]]
    assert np.all(rw.target[mid] == -1)


# ------------------------------------------------ planted mistakes are caught
def test_planted_sign_error_is_caught(tmp_path):
    """Compile a copy of the oracle with one sign flipped in the substitution
    update and check that the dense-solve pin rejects it."""
    import ctypes as C
    import os
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    bad = src.replace("s->wval[sk] = s->wval[sk] - m * v[p];", "s->wval[sk] = s->wval[sk] + m * v[p];")
    assert bad != src
    p = tmp_path / "bad.c"
    p.write_text(bad)
    so = tmp_path / "libbad.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", str(p), "-o", str(so), "-lm"])
    good_lib, good_path = oracle._lib, oracle._LIB_PATH
    try:
        oracle._lib = None
        oracle._LIB_PATH = str(so)
        oracle.build = lambda force=False: str(so)  # noqa: E731
        m = gen.bidiagonal(70, 3)
        lv = oracle.levels(m)
        rw = oracle.rewrite(m, THIN_ROWS, 32, 4.0, 0, None, lv)
        with pytest.raises(AssertionError):
            check_rewrite_invariants(m, rw, lv, THIN_ROWS, 32, 4.0, 0)
    finally:
        import importlib
        importlib.reload(oracle)
        oracle._lib, oracle._LIB_PATH = good_lib, good_path
    del C


# ------------------------------------------------- strategies of Sec. III / IV
def test_standin_generators_match_published_statistics():
    # lung2 / torso2 stand-ins (Sec. IV, Table I): sizes, level counts and the
    # share of 2-row levels are the published ones; nnz within 1 %
    m = gen.lung2_like(0)
    lv = oracle.levels(m)
    w = np.diff(lv.level_ptr)
    assert m.n == 109_460 and lv.nlev == 479 and int((w == 2).sum()) == 453
    assert abs(m.nnz - 492_564) <= 0.01 * 492_564
    m = gen.torso2_like(0)
    lv = oracle.levels(m)
    w = np.diff(lv.level_ptr)
    assert m.n == 115_967 and lv.nlev == 513
    assert abs(m.nnz - 1_033_473) <= 0.01 * 1_033_473
    peak = int(np.argmax(w))
    assert np.all(np.diff(w[:peak]) >= 0) and np.all(np.diff(w[peak + 1:]) <= 0)  # triangular profile


def test_manual_preset_on_the_lung2_standin_closed_form():
    # Sec. IV: the levels cheaper than avgLevelCost are grouped ten at a time,
    # nine rewritten into the first. On the lung2 stand-in these are exactly
    # the 453 two-row levels after the 26 fat ones, so the result has
    # 26 + ceil(453 / 10) levels, 2 * (453 - 46) rows move, each by at most 9
    # levels, and each moved row goes to the first level of its group of ten
    m = gen.lung2_like(0)
    lv = oracle.levels(m)
    c = oracle.level_costs(m, lv)
    thin = c.cost.astype(np.float64) < c.avg
    thin[0] = False
    assert np.array_equal(np.flatnonzero(thin), np.arange(26, 479))
    rank = np.cumsum(thin) - 1
    mask = (thin & (rank % 10 != 0)).astype(np.uint8)
    rw = oracle.rewrite(m, THIN_COST, 1e300, 0.0, 9, mask=mask, lv=lv)
    st = oracle.rewrite_stats(m, rw, lv)
    assert st["nlev_after"] == 26 + 46 and st["rows_rewritten"] == 2 * (453 - 46) and st["max_distance"] == 9
    lev = lv.row_level
    moved = rw.target >= 0
    assert np.array_equal(moved, mask[lev].astype(bool))
    assert np.array_equal(rw.target[moved], 26 + 10 * ((lev[moved] - 26) // 10))


def test_manual_distance_ten_preset_on_a_chain():
    # the comparison approach of Sec. IV: every 9 levels go into the 10th. On a
    # bidiagonal chain (one row per level) with no cost or fill limit, row r
    # moves to level 10 * (r // 10) and L' keeps one dependency per moved row
    n = 45
    m = gen.bidiagonal(n, 5)
    lv = oracle.levels(m)
    mask = (np.arange(lv.nlev) % 10 != 0).astype(np.uint8)
    rw = oracle.rewrite(m, THIN_COST, 1e300, 0.0, 9, mask=mask, lv=lv)
    r = np.arange(n)
    want = np.where(r % 10 == 0, -1, 10 * (r // 10))
    assert np.array_equal(rw.target, want)
    assert rw.max_distance == 9
    lv2 = oracle.levels(rw.lp)
    assert lv2.nlev == (n + 9) // 10
    # every moved row now reads the row just before its group's target (or nothing in group 0)
    for x in range(n):
        cols = rw.lp_col[rw.lp_ptr[x]:rw.lp_ptr[x + 1] - 1].tolist()
        if x % 10 == 0:
            assert cols == ([x - 1] if x else [])
        else:
            g = 10 * (x // 10)
            assert cols == ([g - 1] if g else [])


# ------------------------------------------------ row constraints of Sec. III.A
def _dense_chains(lengths, extra=()):
    """Lower matrix of independent bidiagonal chains of the given lengths, in
    order, plus extra (row, column) dependencies."""
    n = int(sum(lengths))
    a = np.zeros((n, n))
    o = 0
    for L in lengths:
        for i in range(o + 1, o + L):
            a[i, i - 1] = -0.5
        o += L
    for r, c in extra:
        a[r, c] = 0.25
    for i in range(n):
        a[i, i] = 1.0 + np.abs(a[i, :i]).sum()
    return gen.from_dense_lower(a)


def _heights(m):
    """Longest path from each row to a row nothing depends on: the levels of
    the reversed DAG (row i <-> n-1-i, dependencies transposed)."""
    n = m.n
    L = m.to_scipy().tocoo()
    off = L.row != L.col
    R = sp.coo_matrix((L.data[off], (n - 1 - L.col[off], n - 1 - L.row[off])), shape=(n, n)).tolil()
    R.setdiag(1.0)
    rc = R.tocsr()
    rc.sort_indices()
    mr = gen.Csr(n, rc.indptr.astype(np.int32), rc.indices.astype(np.int32), rc.data, "reversed")
    return oracle.levels(mr).row_level[::-1].copy()


def _scan_replay_rc(m, lv, rw, thin_metric, thr, fill_cap, max_distance, alpha, beta, crit):
    """Every decision re-derived from the definitions: the would-be row from
    reachability (B = current level >= target), the stopping tests first
    (budget, fill, distance: refuse and restart at this level with its unmoved
    rows), then the row constraints (leave the row and go on)."""
    c = oracle.level_costs(m, lv)
    W = thr if (thin_metric == THIN_ROWS or thr > 0) else c.avg
    nnz_l = np.diff(m.row_ptr)
    oncrit = lv.row_level + _heights(m) == lv.nlev - 1
    cur = lv.row_level.copy()
    t, size, cost, skipped = 0, c.rows[0], c.cost[0], 0
    for l in range(1, lv.nlev):
        src = c.rows[l] < W if thin_metric == THIN_ROWS else c.cost[l] < W
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        if not src:
            assert np.all(rw.target[rows] == -1)
            t, size, cost = l, c.rows[l], c.cost[l]
            continue
        for r in rows:
            _, A = _reach(m, r, cur >= t)
            nnz_new = len(A) + 1
            ok = (size + 1 <= W) if thin_metric == THIN_ROWS else (cost + 2 * nnz_new - 1 <= W)
            if fill_cap > 0:
                ok = ok and nnz_new <= fill_cap * nnz_l[r]
            if max_distance > 0:
                ok = ok and l - t <= max_distance
            if not ok:
                assert rw.target[r] == -1
                t = l
                left = [q for q in rows if cur[q] == l]
                size, cost = len(left), int(np.sum(2 * nnz_l[left] - 1))
                break
            skip = (alpha > 0 and len(A) >= alpha) or (beta > 0 and len(A) > 0 and max(A) - min(A) >= beta) or \
                (crit and not oncrit[r])
            if skip:
                assert rw.target[r] == -1
                skipped += 1
                continue
            assert rw.target[r] == t
            cur[r] = t
            size += 1
            cost += 2 * nnz_new - 1
    assert skipped == rw.rows_skipped


def test_indegree_limit_on_a_chain():
    # a 40-row chain under the 8-row rule: rows moved into level 0 keep no
    # dependency, later groups keep one (the row before their target). With
    # indegree < 1 only rows 1..7 move; row 8 is refused by the budget and
    # becomes the target; rows 9..39 are left in place
    m = gen.bidiagonal(40, 3)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, THIN_ROWS, 8, 0.0, 0, None, lv, max_indegree=1)
    want = np.full(40, -1)
    want[1:8] = 0
    assert np.array_equal(rw.target, want)
    assert rw.rows_rewritten == 7 and rw.rows_skipped == 31
    assert oracle.levels(rw.lp).nlev == 33
    # indegree < 2 admits every move the unconstrained scan makes
    free = oracle.rewrite(m, THIN_ROWS, 8, 0.0, 0, None, lv)
    rw2 = oracle.rewrite(m, THIN_ROWS, 8, 0.0, 0, None, lv, max_indegree=2)
    assert np.array_equal(rw2.target, free.target) and rw2.rows_skipped == 0
    assert np.array_equal(rw2.lp_col, free.lp_col) and np.array_equal(rw2.t_val, free.t_val)


def test_critical_path_limit_on_two_chains():
    # a 30-row chain beside a 10-row chain: only the long chain lies on a
    # longest path, so only its rows move (all into level 0 under a 64-row
    # budget) and the short chain's 9 movable rows stay
    m = _dense_chains([30, 10])
    lv = oracle.levels(m)
    assert lv.nlev == 30
    rw = oracle.rewrite(m, THIN_ROWS, 64, 0.0, 0, None, lv, critical_only=True)
    want = np.full(40, -1)
    want[1:30] = 0
    assert np.array_equal(rw.target, want)
    assert rw.rows_skipped == 9
    free = oracle.rewrite(m, THIN_ROWS, 64, 0.0, 0, None, lv)
    assert free.rows_rewritten == 38


def test_spread_limit_on_a_chain_reading_row0():
    # rows 2..39 read the row before and row 0. Under the 8-row rule group k
    # (rows 8k+1..8k+7, target level 8k) keeps dependencies {8k-1, 0}: span
    # 8k-1. Span < 10 admits groups 0 and 1; row 16 is refused by the budget
    # and becomes the target; rows 17..39 are left in place
    m = _dense_chains([40], extra=[(r, 0) for r in range(2, 40)])
    lv = oracle.levels(m)
    assert lv.nlev == 40
    rw = oracle.rewrite(m, THIN_ROWS, 8, 0.0, 0, None, lv, max_spread=10)
    want = np.full(40, -1)
    want[1:8] = 0
    want[9:16] = 8
    assert np.array_equal(rw.target, want)
    assert rw.rows_skipped == 23
    lcols = rw.lp_col[rw.lp_ptr[12]:rw.lp_ptr[13] - 1].tolist()
    assert lcols == [0, 7]


RC_CASES = [
    (THIN_ROWS, 6, 0.0, 0, 2, 0, False),
    (THIN_ROWS, 8, 4.0, 0, 0, 6, False),
    (THIN_ROWS, 8, 0.0, 3, 0, 0, True),
    (THIN_COST, 0.0, 0.0, 0, 3, 12, True),
    (THIN_COST, 40.0, 3.0, 0, 0, 0, True),
]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("case", RC_CASES)
def test_row_constraints_random(seed, case):
    # scan decisions re-derived from the definitions, and the rewritten system
    # still exact (L' = T L, unmoved rows untouched, same x)
    rng = np.random.default_rng(300 + seed)
    m = gen.window_random(int(rng.integers(20, 60)), 40 + seed, window=int(rng.integers(2, 9)),
                          draws=int(rng.integers(1, 4)))
    lv = oracle.levels(m)
    tm, thr, cap, md, alpha, beta, crit = case
    rw = oracle.rewrite(m, tm, thr, cap, md, None, lv, max_indegree=alpha, max_spread=beta, critical_only=crit)
    check_rewrite_invariants(m, rw, lv, tm, thr, cap, md)
    _scan_replay_rc(m, lv, rw, tm, thr, cap, md, alpha, beta, crit)


def _same_rewrite(a, b):
    for f in ("lp_ptr", "lp_col", "lp_val", "t_ptr", "t_col", "t_val", "target"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert (a.rows_rewritten, a.max_distance, a.steps, a.rows_skipped) == \
        (b.rows_rewritten, b.max_distance, b.steps, b.rows_skipped)


def _segments(m, lv, tm, thr, mask=None):
    c = oracle.level_costs(m, lv)
    rows = np.diff(lv.level_ptr)
    cost = c.cost
    W = thr if not (tm == THIN_COST and thr <= 0) else c.total / lv.nlev
    src = mask.astype(bool) if mask is not None else ((rows < W) if tm == THIN_ROWS else (cost < W))
    src[0] = False
    return int(np.sum(~src))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("case", RC_CASES)
def test_both_ends_equals_forward(seed, case):
    """The scan taken alternately from the first and the last segment (level 0
    and each non-source level start one) gives the forward scan's result, which
    the replay re-derives from the definitions: a segment's decisions depend on
    nothing outside it."""
    rng = np.random.default_rng(500 + seed)
    m = gen.window_random(int(rng.integers(40, 120)), 60 + seed, window=int(rng.integers(2, 9)),
                          draws=int(rng.integers(1, 4)))
    lv = oracle.levels(m)
    tm, thr, cap, md, alpha, beta, crit = case
    kw = dict(max_indegree=alpha, max_spread=beta, critical_only=crit)
    fwd = oracle.rewrite(m, tm, thr, cap, md, None, lv, **kw)
    both = oracle.rewrite(m, tm, thr, cap, md, None, lv, both_ends=True, **kw)
    _same_rewrite(fwd, both)
    _scan_replay_rc(m, lv, both, tm, thr, cap, md, alpha, beta, crit)


@pytest.mark.parametrize("mk", [lambda: gen.stencil2d_chain(10, 60, 1), lambda: gen.stencil3d_tail(4, 30, 4),
                                lambda: gen.powerlaw(800, 9, w_loc=16, nseg=2, seglen=25),
                                lambda: gen.torso2_like(n=6000, nlev=120)])
def test_both_ends_equals_forward_structured(mk):
    m = mk()
    lv = oracle.levels(m)
    w = max(2, int(np.median(np.diff(lv.level_ptr))) + 1)  # about half the levels thin
    for tm, thr, cap in [(THIN_ROWS, w, 4.0), (THIN_COST, 0.0, 0.0)]:
        assert _segments(m, lv, tm, thr) >= 3  # several segments, so the order differs
        fwd = oracle.rewrite(m, tm, thr, cap, 0, None, lv)
        both = oracle.rewrite(m, tm, thr, cap, 0, None, lv, both_ends=True)
        _same_rewrite(fwd, both)
    rng = np.random.default_rng(3)
    mask = (rng.random(lv.nlev) < 0.7).astype(np.uint8)
    fwd = oracle.rewrite(m, THIN_ROWS, 16, 4.0, 0, mask, lv)
    both = oracle.rewrite(m, THIN_ROWS, 16, 4.0, 0, mask, lv, both_ends=True)
    _same_rewrite(fwd, both)
    _scan_replay(m, lv, both, THIN_ROWS, 16, 4.0, 0, mask)


def _with_planted_oracle(tmp_path, old, new, check):
    """Run check() against a copy of the oracle compiled with one planted
    change (old -> new in oracle.c); the good oracle is restored afterwards."""
    import os
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    bad = src.replace(old, new)
    assert bad != src
    p = tmp_path / "bad.c"
    p.write_text(bad)
    so = tmp_path / "libbad.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", str(p), "-o", str(so), "-lm"])
    good_lib, good_path = oracle._lib, oracle._LIB_PATH
    try:
        oracle._lib = None
        oracle._LIB_PATH = str(so)
        oracle.build = lambda force=False: str(so)  # noqa: E731
        check()
    finally:
        import importlib
        importlib.reload(oracle)
        oracle._lib, oracle._LIB_PATH = good_lib, good_path


def test_planted_two_ended_order_error_is_caught(tmp_path):
    """A two-ended order that takes one segment twice and skips another (an
    off-by-one from the end) must fail the equality with the forward scan."""
    m = gen.window_random(120, 61, window=5, draws=2)
    lv = oracle.levels(m)
    fwd = oracle.rewrite(m, THIN_COST, 0.0, 0.0, 0, None, lv)

    def check():
        assert _segments(m, lv, THIN_COST, 0.0) >= 3
        both = oracle.rewrite(m, THIN_COST, 0.0, 0.0, 0, None, lv, both_ends=True)
        with pytest.raises(AssertionError):
            _same_rewrite(fwd, both)

    _with_planted_oracle(tmp_path, "(k % 2 == 0 ? k / 2 : nseg - 1 - k / 2)", "(k % 2 == 0 ? k / 2 : nseg - k / 2 - (k == 1))",
                         check)


# ------------------------------------------------ per-level budgets and caps
def test_per_level_budget_bidiagonal_closed_form():
    """Bidiagonal, every level one row and a source. Rows of levels below 50
    may fill a target to 5 rows, rows of levels 50 and above to 20: targets
    0, 5, ..., 45 take five rows each; target 45 then takes rows 50..64 (its
    size 5 grows to 20 under the larger budget), and 65 and 85 start groups of
    twenty. Worked out by hand from the scan's definition."""
    m = gen.bidiagonal(100, 5)
    lv = oracle.levels(m)
    budget = np.where(np.arange(lv.nlev) < 50, 5, 20).astype(np.int32)
    rw = oracle.rewrite(m, THIN_ROWS, 1e9, 0.0, 0, None, lv, level_budget=budget)
    want = np.empty(100, np.int64)
    for r in range(100):
        want[r] = 5 * (r // 5) if r < 50 else (45 if r < 65 else (65 if r < 85 else 85))
    got = np.where(rw.target >= 0, rw.target, np.arange(100))
    assert np.array_equal(got, want)
    assert oracle.levels(rw.lp).nlev == len(set(want.tolist()))


def _scan_replay_lv(m, lv, rw, W, cap, budget, lcap):
    """Re-derive every decision of a THIN_ROWS scan with per-level budgets and
    caps from the definition: the rewritten row's size comes from a
    reachability search (nnz(L'[r]) = reachable rows outside B + 1), and a row
    is accepted exactly when the target's size after it fits its level's budget
    and its rewritten size fits its level's cap."""
    c = oracle.level_costs(m, lv)
    cur = _final_cur(lv, rw)
    nnz_l = np.diff(m.row_ptr)
    t, size = 0, c.rows[0]
    for l in range(1, lv.nlev):
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        if not c.rows[l] < W:
            assert np.all(rw.target[rows] == -1)
            t, size = l, c.rows[l]
            continue
        Wl = budget[l] if budget[l] > 0 else W
        capl = float(lcap[l]) if lcap[l] > 0 else cap
        for i, r in enumerate(rows):
            _, A = _reach(m, r, cur >= t)
            ok = size + 1 <= Wl and (capl <= 0 or len(A) + 1 <= capl * nnz_l[r])
            assert (rw.target[r] == t) == ok, (l, r, t)
            if ok:
                size += 1
            else:
                assert np.all(rw.target[rows[i:]] == -1)
                t, size = l, len(rows) - i
                break


@pytest.mark.parametrize("seed", range(6))
def test_per_level_budget_and_cap_replay(seed):
    rng = np.random.default_rng(700 + seed)
    m = gen.window_random(int(rng.integers(200, 600)), 800 + seed, window=int(rng.integers(3, 12)), draws=3)
    lv = oracle.levels(m)
    budget = rng.choice([0, 4, 8, 16, 32], size=lv.nlev).astype(np.int32)
    lcap = rng.choice([0.0, 1.5, 2.0, 4.0, 8.0], size=lv.nlev).astype(np.float32)
    W, cap = 12, 3.0
    rw = oracle.rewrite(m, THIN_ROWS, W, cap, 0, None, lv, level_budget=budget, level_cap=lcap)
    check_rewrite_invariants(m, rw, lv, THIN_ROWS, W, 0.0, 0)
    _scan_replay_lv(m, lv, rw, W, cap, budget, lcap)
    assert rw.rows_rewritten > 0


@pytest.mark.parametrize("old,new", [
    ("const double Wl = (thin_metric == 0 && lv_budget && lv_budget[l] > 0) ? (double)lv_budget[l] : W;",
     "const double Wl = (thin_metric == 0 && lv_budget && lv_budget[t] > 0) ? (double)lv_budget[t] : W;"),
    ("const double capl = (lv_cap && lv_cap[l] > 0.0f) ? (double)lv_cap[l] : fill_cap;",
     "const double capl = (lv_cap && lv_cap[t] > 0.0f) ? (double)lv_cap[t] : fill_cap;")])
def test_planted_per_level_error_is_caught(tmp_path, old, new):
    """Taking the target's budget or cap instead of the source level's fails
    the replay."""
    rng = np.random.default_rng(703)
    m = gen.window_random(400, 803, window=6, draws=3)

    def check():
        lv = oracle.levels(m)
        budget = rng.choice([0, 4, 8, 16, 32], size=lv.nlev).astype(np.int32)
        lcap = rng.choice([0.0, 1.5, 2.0, 4.0, 8.0], size=lv.nlev).astype(np.float32)
        rw = oracle.rewrite(m, THIN_ROWS, 12, 3.0, 0, None, lv, level_budget=budget, level_cap=lcap)
        with pytest.raises(AssertionError):
            _scan_replay_lv(m, lv, rw, 12, 3.0, budget, lcap)

    _with_planted_oracle(tmp_path, old, new, check)


@pytest.mark.parametrize("fill", ["same", "zero"])
def test_uniform_per_level_values_equal_plain_rewrite(fill):
    """Per-level budgets and caps equal to the rewrite's own (or 0, meaning
    the rewrite's own) give the plain rewrite bit for bit."""
    m = gen.window_random(700, 907, window=8, draws=3)
    lv = oracle.levels(m)
    W, cap = 16, 3.0
    budget = np.full(lv.nlev, W if fill == "same" else 0, np.int32)
    lcap = np.full(lv.nlev, cap if fill == "same" else 0.0, np.float32)
    a = oracle.rewrite(m, THIN_ROWS, W, cap, 0, None, lv)
    b = oracle.rewrite(m, THIN_ROWS, W, cap, 0, None, lv, level_budget=budget, level_cap=lcap)
    assert a.rows_rewritten > 0
    assert np.array_equal(a.target, b.target)
    assert np.array_equal(a.lp.row_ptr, b.lp.row_ptr) and np.array_equal(a.lp.col, b.lp.col)
    assert np.array_equal(a.lp.val, b.lp.val)
    assert np.array_equal(a.t_ptr, b.t_ptr) and np.array_equal(a.t_col, b.t_col) and np.array_equal(a.t_val, b.t_val)
