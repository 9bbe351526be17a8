"""GPU parity of sptrsv_rewrite against the oracle: decisions (targets), the
rewritten patterns and values of L' and T, the re-levelled L', Table I style
statistics, and the solve of the rewritten system, through the C ABI."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev
from tests.test_oracle_rewrite import costmap_matrix
from tests.test_oracle_solve_levels import fig2_matrix

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10


def _cases():
    yield "cfg0", gen.config_matrix(0)[0]
    yield "cfg1_small", gen.config_matrix(1, "small")[0]
    yield "cfg2_small", gen.config_matrix(2, "small")[0]
    yield "cfg4_small", gen.config_matrix(4, "small")[0]
    yield "bidiag", gen.bidiagonal(1000, 5)
    yield "window_ragged", gen.window_random(3001, 4, window=12, draws=3)


MATS = list(_cases())
OPTS = {
    "rows32_cap4": dict(thin_metric=0, thin_threshold=32, fill_cap=4.0, max_distance=0),
    "rows8": dict(thin_metric=0, thin_threshold=8, fill_cap=0.0, max_distance=0),
    "cost_avg": dict(thin_metric=1, thin_threshold=0.0, fill_cap=0.0, max_distance=0),
    "cost_avg_cap3_d4": dict(thin_metric=1, thin_threshold=0.0, fill_cap=3.0, max_distance=4),
    "rows64_d2": dict(thin_metric=0, thin_threshold=64, fill_cap=6.0, max_distance=2),
}


def compare(m, h, st, rw, lv, nrhs=(1, 5)):
    assert st["rows_rewritten"] == rw.rows_rewritten
    assert st["max_distance"] == rw.max_distance
    assert st["target_steps"] == rw.steps
    assert np.array_equal(h.targets().cpu().numpy(), rw.target)
    out = {k: v.cpu().numpy() for k, v in h.rewritten().items()}
    for k in ["lp_ptr", "lp_col", "t_ptr", "t_col"]:
        assert np.array_equal(out[k], getattr(rw, k)), k
    # values: same operations in the same order, no contraction -> bit for bit
    assert np.array_equal(out["lp_val"], rw.lp_val)
    assert np.array_equal(out["t_val"], rw.t_val)
    ost = oracle.rewrite_stats(m, rw, lv)
    for k in ["nlev_before", "nlev_after", "nnz_L", "nnz_Lp", "nnz_T", "total_cost_before", "total_cost_after",
              "avg_level_cost_before", "avg_level_cost_after"]:
        assert st[k] == ost[k], k
    lv2 = oracle.levels(rw.lp)
    lp, lr, rl = h.levels(sp.REWRITTEN)
    assert np.array_equal(lp.cpu().numpy(), lv2.level_ptr)
    assert np.array_equal(lr.cpu().numpy(), lv2.level_rows)
    assert np.array_equal(rl.cpu().numpy(), lv2.row_level)
    for k in nrhs:
        b = gen.rhs(m, k)
        xr = oracle.solve(m, b)
        x = h.solve(to_dev(b), which=sp.REWRITTEN)
        h.check()
        assert oracle.relerr(x.cpu().numpy(), xr) <= TOL


@pytest.mark.parametrize("name", [n for n, _ in MATS])
@pytest.mark.parametrize("opt", list(OPTS))
def test_rewrite_parity(name, opt):
    m = dict(MATS)[name]
    o = OPTS[opt]
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(**o)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, o["thin_metric"], o["thin_threshold"], o["fill_cap"], o["max_distance"], None, lv)
    compare(m, h, st, rw, lv)


@pytest.mark.parametrize("seed", range(3))
def test_rewrite_with_mask(seed):
    m = gen.config_matrix(2, "small")[0]
    lv = oracle.levels(m)
    rng = np.random.default_rng(seed)
    mask = (rng.random(lv.nlev) < 0.5).astype(np.uint8)
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 32, 4.0, 0, mask=to_dev(mask))
    rw = oracle.rewrite(m, 0, 32, 4.0, 0, mask, lv)
    compare(m, h, st, rw, lv, nrhs=(1,))


def test_fig2_and_costmap_on_gpu():
    m = fig2_matrix()
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 100, 0.0, 0, mask=to_dev(np.array([0, 1, 1], np.uint8)))
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, 0, 100, 0.0, 0, np.array([0, 1, 1], np.uint8), lv)
    compare(m, h, st, rw, lv, nrhs=(1,))
    assert st["nlev_after"] == 1
    m = costmap_matrix()
    h = sp.Handle()
    h.analyze(*dev(m))
    mask = np.array([0, 0, 1, 1, 1], np.uint8)
    st = h.rewrite(1, 22.0, 0.0, 0, mask=to_dev(mask))
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, 1, 22.0, 0.0, 0, mask, lv)
    compare(m, h, st, rw, lv, nrhs=(1,))
    assert st["nlev_after"] == 3 and st["rows_rewritten"] == 5


def test_config1_full_naive():
    m = gen.config_matrix(1)[0]
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 32, 4.0, 0)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, 0, 32, 4.0, 0, None, lv)
    compare(m, h, st, rw, lv, nrhs=(1,))
    assert st["nlev_before"] == 21999 and st["nlev_after"] == 4826


def test_rewrite_long_rows_use_global_workspace():
    # without a fill cap and with a large budget, rewritten rows outgrow the
    # per-wave LDS workspace and take the global-memory path
    m = gen.window_random(1500, 7, window=40, draws=6)
    lv = oracle.levels(m)
    mask = np.ones(lv.nlev, np.uint8)
    mask[0] = 0
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 1e9, 0.0, 0, mask=to_dev(mask))
    rw = oracle.rewrite(m, 0, 1e9, 0.0, 0, mask, lv)
    assert int(np.max(np.diff(rw.t_ptr))) > 600  # exceeds the LDS workspace
    compare(m, h, st, rw, lv, nrhs=(1,))


def test_rewrite_errors():
    h = sp.Handle()
    with pytest.raises(sp.SptrsvError) as ei:
        h.rewrite()
    assert ei.value.name == "STATE"
    m = gen.config_matrix(0)[0]
    h.analyze(*dev(m))
    with pytest.raises(sp.SptrsvError) as ei:
        h.rewrite(thin_metric=5)
    assert ei.value.name == "ARG"


@pytest.mark.parametrize("w", [4, 8, 40, 130])
def test_b_transform_row_lengths(w):
    # Rows of T of every length class the b-transform distinguishes: on a chain
    # under the W-row rule with no fill cap, a target takes W - 1 moved rows and
    # T's rows hold 1 .. W - 1 off-diagonals (averages about 2, 4, 20 and 64,
    # so a thread per row and 4-, 16- and 64-lane groups). Strided b and x, 1
    # and 3 right-hand sides, n not a multiple of anything
    m = gen.bidiagonal(2011, 7)
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, w, 0.0, 0)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, 0, w, 0.0, 0, None, lv)
    assert st["nnz_T"] == int(rw.t_ptr[-1])
    for k in (1, 3):
        b = gen.rhs(m, k)
        xr = oracle.solve(m, b)
        bd = torch.zeros((k, m.n + 13), dtype=torch.float64, device="cuda")
        bd[:, :m.n] = to_dev(b.reshape(k, m.n))
        xd = torch.full((k, m.n + 5), float("nan"), dtype=torch.float64, device="cuda")
        bb, xx = bd[:, :m.n], xd[:, :m.n]
        if k == 1:
            bb, xx = bb[0], xx[0]
        h.solve(bb, sp.REWRITTEN, xx)
        h.check()
        assert oracle.relerr(xd[:, :m.n].cpu().numpy().reshape(k, m.n), xr.reshape(k, m.n)) <= TOL
        assert torch.isnan(xd[:, m.n:]).all()  # nothing written past each column


# ---------------------------------------------- row constraints (Sec. III.A)
def _chains(lengths, extra=()):
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


RC_MATS = [
    ("bidiag40", lambda: gen.bidiagonal(40, 3)),
    ("two_chains", lambda: _chains([30, 10])),
    ("chain_row0", lambda: _chains([40], extra=[(r, 0) for r in range(2, 40)])),
    ("window_ragged", lambda: gen.window_random(3001, 4, window=12, draws=3)),
    ("cfg1_small", lambda: gen.config_matrix(1, "small")[0]),
    ("cfg2_small", lambda: gen.config_matrix(2, "small")[0]),
]
RC_OPTS = {
    "alpha1": dict(thin_metric=0, thin_threshold=8, fill_cap=0.0, max_distance=0, max_indegree=1),
    "alpha3_cap4": dict(thin_metric=0, thin_threshold=32, fill_cap=4.0, max_distance=0, max_indegree=3),
    "beta10": dict(thin_metric=0, thin_threshold=8, fill_cap=0.0, max_distance=0, max_spread=10),
    "crit": dict(thin_metric=0, thin_threshold=64, fill_cap=0.0, max_distance=0, critical_only=True),
    "cost_all": dict(thin_metric=1, thin_threshold=0.0, fill_cap=0.0, max_distance=0, max_indegree=4,
                     max_spread=200, critical_only=True),
}


@pytest.mark.parametrize("name", [n for n, _ in RC_MATS])
@pytest.mark.parametrize("opt", list(RC_OPTS))
def test_row_constraints_parity(name, opt):
    m = dict(RC_MATS)[name]()
    o = RC_OPTS[opt]
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(**o)
    lv = oracle.levels(m)
    rw = oracle.rewrite(m, o["thin_metric"], o["thin_threshold"], o["fill_cap"], o["max_distance"], None, lv,
                        max_indegree=o.get("max_indegree", 0), max_spread=o.get("max_spread", 0),
                        critical_only=o.get("critical_only", False))
    assert st["rows_skipped"] == rw.rows_skipped
    compare(m, h, st, rw, lv, nrhs=(1, 3))


def test_row_constraints_with_global_workspace():
    # rows whose rewritten form overflows the LDS workspace are evaluated again
    # in the global one; some of them are then held by a constraint
    # (levels 0 and 10 are the targets; rows beyond level 10 keep 11
    # dependencies on levels before it, so indegree < 11 holds them)
    m = gen.window_random(1500, 7, window=40, draws=6)
    lv = oracle.levels(m)
    mask = np.ones(lv.nlev, np.uint8)
    mask[0] = 0
    mask[10] = 0
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 1e9, 0.0, 0, mask=to_dev(mask), max_indegree=11)
    rw = oracle.rewrite(m, 0, 1e9, 0.0, 0, mask, lv, max_indegree=11)
    assert rw.rows_skipped > 1000 and rw.rows_rewritten > 0
    assert st["rows_skipped"] == rw.rows_skipped
    compare(m, h, st, rw, lv, nrhs=(1,))


def test_row_constraint_errors():
    m = gen.bidiagonal(50, 1)
    h = sp.Handle()
    h.analyze(*dev(m))
    for bad in (dict(max_indegree=-1), dict(max_spread=-5)):
        with pytest.raises(sp.SptrsvError):
            h.rewrite(sp.THIN_ROWS, 8.0, 0.0, 0, **bad)


def _wide_row_matrix(k=17000):
    # rows 0..k-1 stand alone; row k reads all of them; row k+1 reads all of
    # them and row k: rewriting either row takes more than 2^14 workspace
    # entries, past the per-wave retry region, into the full workspace
    rng = np.random.default_rng(5)
    cols = [np.array([i]) for i in range(k)]
    cols.append(np.arange(k + 1))
    cols.append(np.arange(k + 2))
    rp = np.zeros(k + 3, np.int64)
    rp[1:] = np.cumsum([c.size for c in cols])
    ci = np.concatenate(cols).astype(np.int32)
    va = rng.uniform(-1.0, 1.0, ci.size) / k
    va[rp[1:] - 1] = 2.0
    return gen.Csr(k + 2, rp.astype(np.int32), ci, va, "wide_rows")


@pytest.mark.parametrize("held", [False, True])
def test_rewrite_rows_past_the_retry_region(held):
    m = _wide_row_matrix()
    lv = oracle.levels(m)
    assert lv.nlev == 3
    h = sp.Handle()
    h.analyze(*dev(m))
    if held:  # level 1 is a target: row k+1 keeps k columns, indegree < 100 holds it
        mask = np.array([0, 0, 1], np.uint8)
        st = h.rewrite(0, 1e9, 0.0, 0, mask=to_dev(mask), max_indegree=100)
        rw = oracle.rewrite(m, 0, 1e9, 0.0, 0, mask, lv, max_indegree=100)
        assert rw.rows_skipped == 1 and rw.rows_rewritten == 0
    else:
        st = h.rewrite(0, 1e9, 0.0, 0)
        rw = oracle.rewrite(m, 0, 1e9, 0.0, 0, None, lv)
        assert rw.rows_rewritten == 2 and int(np.max(np.diff(rw.t_ptr))) > 1 << 14
    assert st["rows_skipped"] == rw.rows_skipped
    compare(m, h, st, rw, lv, nrhs=(1,))


SEG_CASES = {
    "cfg2_rows32": (lambda: gen.config_matrix(2, "small")[0], OPTS["rows32_cap4"]),
    "cfg4_cost": (lambda: gen.config_matrix(4, "small")[0], OPTS["cost_avg"]),
    "window_rc": (lambda: gen.window_random(3001, 4, window=12, draws=3), RC_OPTS["cost_all"]),
    "torso_cost": (lambda: gen.torso2_like(n=20000, nlev=200), OPTS["cost_avg_cap3_d4"]),
    "cfg1_rows8": (lambda: gen.config_matrix(1, "small")[0], OPTS["rows8"]),
}


@pytest.mark.parametrize("workers", [2, 3, 16])
@pytest.mark.parametrize("case", list(SEG_CASES))
def test_scan_from_both_ends_parity(case, workers):
    """Several workgroups take the scan's segments from both ends of the level
    order at once; every decision, pattern and value equals the oracle's."""
    from tests.test_oracle_rewrite import _segments
    mk, o = SEG_CASES[case]
    m = mk()
    lv = oracle.levels(m)
    assert _segments(m, lv, o["thin_metric"], o["thin_threshold"]) >= workers
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(**o, scan_workers=workers)
    rw = oracle.rewrite(m, o["thin_metric"], o["thin_threshold"], o["fill_cap"], o["max_distance"], None, lv,
                        max_indegree=o.get("max_indegree", 0), max_spread=o.get("max_spread", 0),
                        critical_only=o.get("critical_only", False), both_ends=True)
    assert st["rows_skipped"] == rw.rows_skipped
    compare(m, h, st, rw, lv, nrhs=(1,))


def test_scan_from_both_ends_with_mask_and_global_workspace():
    # segments start at the unmasked levels; rows that overflow the LDS
    # workspace take each workgroup's own global one
    m = gen.window_random(1500, 7, window=40, draws=6)
    lv = oracle.levels(m)
    mask = np.ones(lv.nlev, np.uint8)
    mask[[0, 10, 40, 41, 90]] = 0
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(0, 1e9, 0.0, 0, mask=to_dev(mask), max_indegree=11, scan_workers=4)
    rw = oracle.rewrite(m, 0, 1e9, 0.0, 0, mask, lv, max_indegree=11, both_ends=True)
    assert rw.rows_rewritten > 0
    assert st["rows_skipped"] == rw.rows_skipped
    compare(m, h, st, rw, lv, nrhs=(1,))


def test_scan_workers_errors():
    m = gen.bidiagonal(50, 1)
    h = sp.Handle()
    h.analyze(*dev(m))
    for bad in (-1, 17):
        with pytest.raises(sp.SptrsvError):
            h.rewrite(sp.THIN_ROWS, 8.0, 0.0, 0, scan_workers=bad)
    st = h.rewrite(sp.THIN_ROWS, 8.0, 0.0, 0, scan_workers=0)  # 0 is one workgroup
    rw = oracle.rewrite(m, sp.THIN_ROWS, 8.0, 0.0, 0)
    assert st["rows_rewritten"] == rw.rows_rewritten


def _hub_matrix(D):
    """Rows 0..D-1 have no dependency (level 0); row D reads all of them (level
    1); row D+1 reads row D (level 2). Rewriting row D toward level 0
    substitutes D rows: its T row needs D entries."""
    rng = np.random.default_rng(21)
    n = D + 2
    off = rng.uniform(-1.0, 1.0, D)
    rp = np.concatenate([np.arange(0, D + 1), [2 * D + 1, 2 * D + 3]]).astype(np.int64)
    col = np.concatenate([np.arange(D), np.arange(D), [D, D, D + 1]]).astype(np.int32)
    val = np.concatenate([np.ones(D), off, [1.0 + np.abs(off).sum(), -0.5, 2.0]])
    return gen.Csr(n, rp.astype(np.int32), col, val, "hub")


def test_rewrite_beyond_the_scan_workspace_is_an_overflow_error():
    """A row whose rewritten form outgrows the scan's per-wave global
    workspace (about 1M entries) is refused with SPTRSV_ERR_OVERFLOW (fill cap
    off); the handle keeps its analysis and has no rewrite."""
    m = _hub_matrix(1_100_000)
    h = sp.Handle()
    h.analyze(*dev(m))
    with pytest.raises(sp.SptrsvError) as e:
        h.rewrite(sp.THIN_ROWS, 1e9, 0.0, 0)
    assert e.value.name == "OVERFLOW"
    b = torch.from_numpy(gen.rhs(m, 1)).cuda()
    x = h.solve(b)
    h.check()
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, b.cpu().numpy())) <= 1e-10
    with pytest.raises(sp.SptrsvError) as e:
        h.solve(b, sp.REWRITTEN)
    assert e.value.name == "STATE"


def _growing_chain(n, ratio):
    """Bidiagonal chain x_i = b_i + ratio x_{i-1} (diagonal 1, off-diagonal
    -ratio): with b = L 1 every x_i is exactly 1, but the rewritten rows carry
    products ratio^k in T, and b' = T b cancels them in floating point."""
    rp = np.concatenate([[0], 1 + 2 * np.arange(n)]).astype(np.int32)
    col = np.concatenate([[0]] + [[i - 1, i] for i in range(1, n)]).astype(np.int32)
    val = np.concatenate([[1.0]] + [[-ratio, 1.0] for _ in range(1, n)])
    return gen.Csr(n, rp, col, val, "chain")


def test_self_check_falls_back_to_the_original_system():
    m = _growing_chain(300, 10.0)
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(sp.THIN_ROWS, 32, 0.0, 0, self_check=1e-8)
    assert st["self_check_failed"] == 1 and st["self_check_err"] > 1e-8
    assert st["rows_rewritten"] == 0 and st["nlev_after"] == st["nlev_before"] == 300
    g = h.rewritten()
    assert np.array_equal(g["lp_ptr"].cpu().numpy(), m.row_ptr) and np.array_equal(g["lp_col"].cpu().numpy(), m.col)
    assert np.array_equal(g["lp_val"].cpu().numpy(), m.val)
    assert np.array_equal(g["t_ptr"].cpu().numpy(), np.arange(m.n + 1))
    assert np.all(g["t_val"].cpu().numpy() == 1.0)
    assert np.all(h.targets().cpu().numpy() == -1)
    one = np.ones((1, m.n))
    b = torch.from_numpy(oracle.spmv(m.row_ptr, m.col, m.val, m.n, one)).cuda()
    x0 = h.solve(b, sp.ORIGINAL)
    x1 = h.solve(b, sp.REWRITTEN)
    h.check()  # the failed check left no error latched
    assert torch.equal(x0, x1)
    assert np.all(x0.cpu().numpy() == 1.0)
    # without the check the rewritten system is far off
    h2 = sp.Handle()
    h2.analyze(*dev(m))
    h2.rewrite(sp.THIN_ROWS, 32, 0.0, 0)
    x2 = h2.solve(b, sp.REWRITTEN)
    assert not np.allclose(x2.cpu().numpy(), 1.0, rtol=1e-8)


def test_self_check_passes_on_a_dominant_matrix():
    m = gen.config_matrix(1, "small")[0]
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(sp.THIN_ROWS, 32, 4.0, 0, self_check=1e-10)
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0)
    assert st["self_check_failed"] == 0 and 0.0 <= st["self_check_err"] <= 1e-12
    assert st["rows_rewritten"] == rw.rows_rewritten


@pytest.mark.parametrize("case", ["window", "cfg1_small", "cfg2_small", "powerlaw_mask"])
def test_per_level_budget_and_cap_parity(case):
    """Per-level row budgets and fill caps (the learned policy's actions):
    rewritten L', T, targets and levels bit for bit against the oracle."""
    rng = np.random.default_rng({"window": 1, "cfg1_small": 2, "cfg2_small": 3, "powerlaw_mask": 4}[case])
    m = {"window": lambda: gen.window_random(4000, 9, window=20, draws=4),
         "cfg1_small": lambda: gen.config_matrix(1, "small")[0],
         "cfg2_small": lambda: gen.config_matrix(2, "small")[0],
         "powerlaw_mask": lambda: gen.powerlaw(30000, 12, w_loc=300, nseg=3, seglen=80)}[case]()
    lv = oracle.levels(m)
    budget = rng.choice([0, 16, 32, 64, 128], size=lv.nlev).astype(np.int32)
    lcap = rng.choice([0.0, 2.0, 4.0, 8.0], size=lv.nlev).astype(np.float32)
    mask = None
    if case == "powerlaw_mask":
        mask = (rng.random(lv.nlev) < 0.7).astype(np.uint8)
        mask[0] = 0
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(sp.THIN_ROWS, 32, 4.0, 0, to_dev(mask) if mask is not None else None,
                   level_budget=to_dev(budget), level_fill_cap=to_dev(lcap))
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32, 4.0, 0, mask, lv, level_budget=budget, level_cap=lcap)
    assert rw.rows_rewritten > 0
    compare(m, h, st, rw, lv, nrhs=(1,))
