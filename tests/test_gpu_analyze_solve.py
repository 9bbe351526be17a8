"""GPU parity: sptrsv_analyze (levels, statistics, validation) and
sptrsv_solve against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu

sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10  # relative error bound on x (normwise, per RHS column)


def _matrices():
    yield "diag", gen.diagonal(100, 1)
    yield "bidiag", gen.bidiagonal(700, 2)
    yield "one", gen.diagonal(1, 3)
    yield "cfg0", gen.config_matrix(0)[0]
    yield "cfg1_small", gen.config_matrix(1, "small")[0]
    yield "cfg2_small", gen.config_matrix(2, "small")[0]
    yield "cfg4_small", gen.config_matrix(4, "small")[0]
    yield "window_ragged", gen.window_random(5003, 9, window=200, draws=7)


MATS = list(_matrices())


@pytest.fixture(scope="module")
def handles():
    out = {}
    for name, m in MATS:
        h = sp.Handle()
        nlev = h.analyze(*dev(m))
        out[name] = (m, h, nlev)
    return out


@pytest.mark.parametrize("name", [n for n, _ in MATS])
def test_levels_bit_exact(handles, name):
    m, h, nlev = handles[name]
    lv = oracle.levels(m)
    assert nlev == lv.nlev
    lp, lr, rl = h.levels()
    assert np.array_equal(lp.cpu().numpy(), lv.level_ptr)
    assert np.array_equal(lr.cpu().numpy(), lv.level_rows)
    assert np.array_equal(rl.cpu().numpy(), lv.row_level)


@pytest.mark.parametrize("name", [n for n, _ in MATS])
def test_level_stats_exact(handles, name):
    m, h, _ = handles[name]
    c = oracle.level_costs(m)
    st = h.level_stats()
    assert np.array_equal(st["rows"].cpu().numpy(), c.rows)
    assert np.array_equal(st["nnz"].cpu().numpy(), c.nnz)
    assert np.array_equal(st["cost"].cpu().numpy(), c.cost)
    assert st["total"] == c.total and st["avg"] == c.avg


SCHEDS = [dict(mode=0), dict(mode=1), dict(mode=2), dict(mode=0, thin_rows=64, wg_threads=256),
          dict(mode=1, lanes_per_row=4), dict(mode=0, thin_rows=300, wg_threads=1024, lanes_per_row=8),
          dict(mode=1, wide_grid=256), dict(mode=0, thin_rows=64, wide_threads=512, wide_grid=1024),
          dict(mode=1, wide_threads=64, wide_grid=3), dict(mode=3),
          dict(mode=4), dict(mode=4, thin_rows=0, wide_threads=128), dict(mode=4, thin_rows=64, wide_threads=512, wide_grid=7)]


@pytest.mark.parametrize("name", [n for n, _ in MATS])
@pytest.mark.parametrize("si", range(len(SCHEDS)))
@pytest.mark.parametrize("nrhs", [1, 3, 40])
def test_solve_parity(handles, name, si, nrhs):
    m, h, _ = handles[name]
    h.set_schedule(**SCHEDS[si])
    b = gen.rhs(m, nrhs)
    xr = oracle.solve(m, b)
    x = h.solve(to_dev(b))
    h.check()
    assert oracle.relerr(x.cpu().numpy(), xr) <= TOL
    h.set_schedule()


def _band(n, k, seed):
    # every row reads the k rows before it: one row per level, min(r, k)
    # in-window dependencies
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for i in range(n):
        lo = max(0, i - k)
        a[i, lo:i] = rng.uniform(-1.0, 1.0, i - lo)
        a[i, i] = 1.0 + np.abs(a[i, lo:i]).sum()
    return gen.from_dense_lower(a, f"band{k}_n{n}")


@pytest.mark.parametrize("k", [3, 6, 12, 24, 40])
@pytest.mark.parametrize("nrhs", [1, 3, 5])
@pytest.mark.parametrize("wg", [256, 1024])
def test_band_chain_parity(k, nrhs, wg):
    # one row per level with up to k in-window dependencies: the overflow
    # records of one-wave windows in several batches, 1 to 5 items per level
    m = _band(301, k, k + 7 * nrhs)
    h = sp.Handle()
    h.analyze(*dev(m))
    h.set_schedule(sp.ORIGINAL, mode=2, wg_threads=wg)
    b = gen.rhs(m, nrhs)
    xr = oracle.solve(m, b)
    bd = to_dev(b)
    x = h.solve(bd if nrhs > 1 else bd.view(-1))
    h.check()
    assert oracle.relerr(x.view(nrhs, -1).cpu().numpy(), xr) <= TOL
    x2 = h.solve(bd if nrhs > 1 else bd.view(-1))
    assert torch.equal(x, x2)


def test_solve_deterministic(handles):
    m, h, _ = handles["cfg2_small"]
    b = to_dev(gen.rhs(m, 2))
    x1 = h.solve(b).clone()
    x2 = h.solve(b)
    assert torch.equal(x1, x2)


def test_ones_solution(handles):
    m, h, _ = handles["cfg1_small"]
    b = m.to_scipy() @ np.ones(m.n)
    x = h.solve(to_dev(b))
    assert float((x - 1).abs().max()) < 1e-12


def test_strided_ld(handles):
    m, h, _ = handles["cfg0"]
    nrhs, ld = 3, m.n + 17
    bb = np.zeros((nrhs, ld))
    bb[:, :m.n] = gen.rhs(m, nrhs)
    xr = oracle.solve(m, bb[:, :m.n])
    B = to_dev(bb)
    X = torch.full((nrhs, ld), 7.0, dtype=torch.float64, device="cuda")
    h.solve(B[:, :m.n], x=X[:, :m.n])
    assert oracle.relerr(X[:, :m.n].cpu().numpy(), xr) <= TOL
    assert torch.all(X[:, m.n:] == 7.0)


def _csr(n, rows):
    rp, ci, v = [0], [], []
    for r in rows:
        for c, x in r:
            ci.append(c)
            v.append(x)
        rp.append(len(ci))
    return gen.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v, np.float64), "t")


BAD = [
    [[(0, 2.0)], [(1, 3.0), (0, 1.0)]],
    [[(0, 2.0)], [(0, 1.0), (0, 1.0), (1, 3.0)]],
    [[(0, 2.0), (1, 1.0)], [(1, 3.0)]],
    [[(0, 2.0)], [(0, 1.0)]],
    [[(0, 0.0)], [(0, 1.0), (1, 3.0)]],
    [[(0, 2.0)], [(0, float("nan")), (1, 3.0)]],
    [[(0, 2.0)], [(1, 3.0), (0, 1.0)], [(3, 1.0), (2, 1.0)]],
]


@pytest.mark.parametrize("rows", BAD)
def test_validation_matches_oracle(rows):
    m = _csr(len(rows), rows)
    expect = oracle.validate(m)
    h = sp.Handle()
    with pytest.raises(sp.SptrsvError) as ei:
        h.analyze(*dev(m))
    assert ei.value.name == expect


def test_bad_row_ptr():
    m = gen.window_random(50, 1)
    rp = m.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]
    h = sp.Handle()
    with pytest.raises(sp.SptrsvError) as ei:
        h.analyze(to_dev(rp), to_dev(m.col), to_dev(m.val))
    assert ei.value.name == "ARG" == oracle.validate(gen.Csr(m.n, rp, m.col, m.val))


def test_state_and_arg_errors(handles):
    m, h, _ = handles["cfg0"]
    b = to_dev(gen.rhs(m, 1)[0])
    with pytest.raises(sp.SptrsvError) as ei:
        h.solve(b, which=sp.REWRITTEN)
    assert ei.value.name == "STATE"
    with pytest.raises(sp.SptrsvError) as ei:
        h.solve(b, x=b)  # aliasing
    assert ei.value.name == "ARG"


@pytest.mark.parametrize("bad", [dict(mode=5), dict(overlap=2), dict(overlap=-1), dict(lanes_per_row=3), dict(wg_threads=300),
                                 dict(mode=4, wide_threads=1024), dict(mode=3, wide_grid=4096), dict(thin_cols=-1)])
def test_bad_schedule_is_refused(handles, bad):
    _, h, _ = handles["cfg0"]
    with pytest.raises(sp.SptrsvError) as ei:
        h.set_schedule(**bad)
    assert ei.value.name == "ARG"
    h.set_schedule()


def test_nonfinite_latched(handles):
    m, h, _ = handles["cfg0"]
    b = gen.rhs(m, 1)[0]
    b[17] = np.nan
    h.solve(to_dev(b))
    with pytest.raises(sp.SptrsvError) as ei:
        h.check()
    assert ei.value.name == "NONFINITE"
    h.check()  # cleared


def test_residual(handles):
    m, h, _ = handles["cfg4_small"]
    b = to_dev(gen.rhs(m, 2))
    x = h.solve(b)
    r = h.residual(b, x)
    assert max(r) < 1e-12


def test_graph_replays(handles):
    m, h, _ = handles["cfg1_small"]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = to_dev(gen.rhs(m, 1))
        x = torch.zeros_like(b)
        gid = h.graph_create(b, x)
        xr = oracle.solve(m, b.cpu().numpy())
        for rep in range(3):
            x.zero_()
            h.graph_launch(gid)
            torch.cuda.synchronize()
            assert oracle.relerr(x.cpu().numpy(), xr) <= TOL
            b2 = b * 2.0  # eager work between replays
            torch.cuda.synchronize()
            del b2


@pytest.mark.parametrize("sched", [dict(mode=1, wide_grid=256), dict(mode=0, thin_rows=16, wide_grid=64),
                                   dict(mode=4, thin_rows=16), dict(mode=4, thin_rows=0, wide_threads=128)])
def test_graph_replays_persistent_wide(handles, sched):
    # the barrier counters of a persistent wide run reset themselves at the end
    # of every launch, so graph replays and eager solves can alternate
    m, h, _ = handles["cfg4_small"]
    h.set_schedule(**sched)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = to_dev(gen.rhs(m, 3))
        x = torch.zeros_like(b)
        gid = h.graph_create(b, x)
        xr = oracle.solve(m, b.cpu().numpy())
        for rep in range(3):
            x.zero_()
            h.graph_launch(gid)
            torch.cuda.synchronize()
            assert oracle.relerr(x.cpu().numpy(), xr) <= TOL
            xe = h.solve(b)
            torch.cuda.synchronize()
            assert torch.equal(xe, x)
    h.check()
    h.set_schedule()


def test_autotune_keeps_parity(handles):
    m, h, _ = handles["cfg2_small"]
    ms = h.autotune(nrhs=1)
    assert ms > 0
    b = gen.rhs(m, 1)
    x = h.solve(to_dev(b))
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, b)) <= TOL
    h.set_schedule()


def test_set_schedule_replaces_tuned(handles):
    m, h, _ = handles["cfg2_small"]
    h.autotune(nrhs=2)
    tuned = h.get_schedule(nrhs=2)
    assert tuned["mode"] in (0, 1, 2, 3)
    assert h.get_schedule(nrhs=1) == dict(mode=0, thin_rows=4096, wg_threads=512, wide_threads=256, lanes_per_row=1,
                                          wide_grid=0, overlap=0, thin_cols=0)
    assert tuned["overlap"] == 0  # the autotuner keeps the transposes out of the chain
    want = dict(mode=0, thin_rows=64, wg_threads=256, wide_threads=128, lanes_per_row=1, wide_grid=0, overlap=0,
                thin_cols=0)
    h.set_schedule(**want)
    assert h.get_schedule(nrhs=2) == want  # an explicit schedule replaces the tuned one
    h.prepare(nrhs=2)
    b = gen.rhs(m, 2)
    x = h.solve(to_dev(b))
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, b)) <= TOL
    h.set_schedule()


def test_empty_matrix():
    h = sp.Handle()
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    nlev = h.analyze(z, torch.zeros(0, dtype=torch.int32, device="cuda"),
                     torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert nlev == 0


def test_syncfree_graph_replays_and_rewrite(handles):
    # the synchronisation-free executor (mode 3): graph replays (its ticket and
    # pending marks are reset by a kernel of the graph), repeated solves give
    # the same bits, and the rewritten system of the chain matrix
    m, h, _ = handles["cfg1_small"]
    h.set_schedule(mode=3)
    b = to_dev(gen.rhs(m, 1))
    xr = oracle.solve(m, b.cpu().numpy())
    x1 = h.solve(b.view(-1))
    x2 = h.solve(b.view(-1))
    h.check()
    assert torch.equal(x1, x2)
    assert oracle.relerr(x1.cpu().numpy(), xr) <= TOL
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x = torch.zeros_like(b)
        gid = h.graph_create(b, x)
        for _ in range(3):
            x.zero_()
            h.graph_launch(gid)
            torch.cuda.synchronize()
            assert oracle.relerr(x.cpu().numpy(), xr) <= TOL
    h.check()
    h.rewrite(sp.THIN_ROWS, 32, 4.0, 0)
    h.set_schedule(sp.REWRITTEN, mode=3)
    for nrhs in (1, 5):
        bb = gen.rhs(m, nrhs)
        x = h.solve(to_dev(bb) if nrhs > 1 else to_dev(bb[0]), sp.REWRITTEN)
        h.check()
        assert oracle.relerr(x.cpu().numpy().reshape(nrhs, -1), oracle.solve(m, bb)) <= TOL
    h.set_schedule(mode=0)


@pytest.mark.parametrize("grid", [1, 16, 2048])
def test_syncfree_grid_sizes(handles, grid):
    # one workgroup still finishes (it takes every ticket in turn)
    m, h, _ = handles["window_ragged"]
    h.set_schedule(mode=3, wide_grid=grid)
    for nrhs in (1, 3):
        b = gen.rhs(m, nrhs)
        x = h.solve(to_dev(b))
        h.check()
        assert oracle.relerr(x.cpu().numpy().reshape(nrhs, -1), oracle.solve(m, b)) <= TOL
    with pytest.raises(sp.SptrsvError) as ei:
        h.set_schedule(mode=3, wide_grid=4096)
    assert ei.value.name == "ARG"
    h.set_schedule(mode=0)


def _long_rows_matrix(n=6000, first=4000, reach=4000, seed=11):
    """Rows first..first+63 (one wave's claim) each read every row below
    `reach` and the row before them, so the whole wave sweeps long rows whose
    last dependency is a lower lane of its own wave; a few later rows read
    hundreds of spread-out rows; the rest are a random window pattern."""
    rng = np.random.default_rng(seed)
    rp, ci, va = [0], [], []
    for r in range(n):
        if first <= r < first + 64:
            cols = list(range(0, reach, 1)) + ([r - 1] if r - 1 >= reach else [])
        elif r >= first + 64 and r % 97 == 0:
            cols = sorted(set(rng.choice(r, size=min(r, 700), replace=False).tolist()))
        else:
            k = min(r, 3)
            cols = sorted(set((r - 1 - rng.integers(0, 40, size=k)).clip(0).tolist())) if r else []
            cols = [c for c in cols if c < r]
        for c in cols:
            ci.append(c)
            va.append(-0.5 / max(1, len(cols)))
        ci.append(r)
        va.append(2.0)
        rp.append(len(ci))
    return gen.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


def test_levels_with_long_rows():
    # rows with more than 256 dependencies left are swept by the whole wave,
    # which steps back while a dependency (here a lower lane of the same wave)
    # is still pending
    m = _long_rows_matrix()
    lv = oracle.levels(m)
    h = sp.Handle()
    nlev = h.analyze(*dev(m))
    assert nlev == lv.nlev
    lp, lr, rl = h.levels()
    assert np.array_equal(rl.cpu().numpy(), lv.row_level)
    assert np.array_equal(lr.cpu().numpy(), lv.level_rows)
    b = gen.rhs(m, 1)
    x = h.solve(to_dev(b))
    h.check()
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, b)) <= TOL
