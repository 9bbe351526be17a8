"""GPU parity of solves with the right-hand sides stored by rows
(sptrsv_solve_rows: entry (i, c) at i * nrhs + c). Against the oracle, and bit
for bit against the column-major solve of the same system and schedule (the
same kernels and order): plain and rewritten systems, the upper and
transposed forms (reversed numbering), every schedule family (the direct path
of thin runs and wide launches, and the copy-by-rows path of persistent,
dataflow and synchronisation-free schedules), one and several right-hand
sides, and hipGraph replays."""
import ctypes

import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")
sptrsv_mod = pytest.importorskip("paper_2206_05843_amd.sptrsv")

TOL = 1e-10
SCHEDS = [dict(mode=0, thin_rows=64, wg_threads=512), dict(mode=0, thin_rows=4096, wg_threads=1024),
          dict(mode=1, wide_threads=128), dict(mode=2, wg_threads=256),
          dict(mode=1, wide_grid=64), dict(mode=3, wide_grid=128), dict(mode=4, thin_rows=64, wide_threads=256),
          dict(mode=0, thin_rows=64, wg_threads=1024, wide_grid=4096, thin_cols=1),
          dict(mode=0, thin_rows=256, wg_threads=512, wide_grid=256, wide_threads=512, thin_cols=2)]
MATS = {"stencil3d_tail": lambda: gen.stencil3d_tail(16, 300, 5), "window": lambda: gen.window_random(3000, 7, 40, 5),
        "cfg2_small": lambda: gen.config_matrix(2, "small")[0]}


@pytest.fixture(scope="module")
def mats():
    return {k: f() for k, f in MATS.items()}


def _oracle(m, b_cols, form):
    return oracle.solve(m, b_cols) if form == sp.LOWER else oracle.solve_form(m, b_cols, form)


@pytest.mark.parametrize("sched", range(len(SCHEDS)))
@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("rewrite", [False, True])
@pytest.mark.parametrize("nrhs", [3, 32])
def test_rows_match_columns_and_oracle(mats, name, rewrite, sched, nrhs):
    m = mats[name]
    print(f"rows: {name} rewrite={rewrite} sched={SCHEDS[sched]} nrhs={nrhs}", flush=True)
    h = sp.Handle()
    h.analyze(*dev(m))
    which = sp.ORIGINAL
    if rewrite:
        h.rewrite(sp.THIN_ROWS, 32, 4.0)
        which = sp.REWRITTEN
    h.set_schedule(which, **SCHEDS[sched])
    b_cols = gen.rhs(m, nrhs)  # (nrhs, n): column c = b_cols[c]
    bc = torch.from_numpy(b_cols).cuda()
    br = bc.t().contiguous()  # (n, nrhs): by rows
    x_cols = h.solve(bc, which)
    h.check()
    x_rows = h.solve_rows(br, which)
    h.check()
    assert torch.equal(x_rows.t(), x_cols)
    assert oracle.relerr(x_rows.t().cpu().numpy(), oracle.solve(m, b_cols)) <= TOL


@pytest.mark.parametrize("form", [sp.UPPER, sp.LOWER_TRANS])
def test_rows_forms(mats, form):
    m = mats["stencil3d_tail"]
    mm = gen.transpose(m) if form == sp.UPPER else m
    h = sp.Handle()
    h.analyze(*dev(mm), form=form)
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    b_cols = gen.rhs(m, 5)
    bc = torch.from_numpy(b_cols).cuda()
    for sched in (SCHEDS[0], SCHEDS[5]):
        h.set_schedule(sp.REWRITTEN, **sched)
        x_cols = h.solve(bc, sp.REWRITTEN)
        x_rows = h.solve_rows(bc.t().contiguous(), sp.REWRITTEN)
        h.check()
        assert torch.equal(x_rows.t(), x_cols)
        assert oracle.relerr(x_cols.cpu().numpy(), _oracle(mm, b_cols, form)) <= TOL


def test_rows_one_rhs_and_errors(mats):
    m = mats["window"]
    h = sp.Handle()
    h.analyze(*dev(m))
    b = torch.from_numpy(gen.rhs(m, 1)[0]).cuda()
    x1 = h.solve(b)
    xr = h.solve_rows(b.view(-1, 1))
    h.check()
    assert torch.equal(xr.view(-1), x1)
    br = torch.from_numpy(gen.rhs(m, 4).T.copy()).cuda()
    with pytest.raises(sp.SptrsvError) as ei:
        h.solve_rows(br, x=br)  # b and x overlap
    assert ei.value.name == "ARG"


def test_rows_graph_replays(mats):
    """Captured once, replayed three times with eager work in between; every
    replay equals the eager column-major solve transposed."""
    m = mats["stencil3d_tail"]
    h = sp.Handle()
    h.analyze(*dev(m))
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    h.set_schedule(sp.REWRITTEN, **SCHEDS[0])
    b_cols = gen.rhs(m, 32)
    bc = torch.from_numpy(b_cols).cuda()
    x_ref = h.solve(bc, sp.REWRITTEN).t().contiguous()
    h.check()
    br = bc.t().contiguous()
    x = torch.zeros_like(br)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        gid = h.graph_create_rows(br, x, sp.REWRITTEN)
        for rep in range(3):
            x.zero_()
            h.graph_launch(gid)
            s.synchronize()
            assert torch.equal(x, x_ref), rep
            y = h.solve(bc, sp.REWRITTEN)
            s.synchronize()
            assert torch.equal(y.t(), x_ref)
    h.check()


def test_rows_level_floor(mats):
    """The level floor of a solve by rows drops the gather and scatter
    launches under the direct schedules and keeps them under the others;
    unknown flag bits are refused."""
    m = mats["window"]
    h = sp.Handle()
    h.analyze(*dev(m))
    costs = h.measure_level_costs()
    h.set_schedule(sp.ORIGINAL, **SCHEDS[0])
    cols = h.level_floor(costs, sp.ORIGINAL, 4)
    rows = h.level_floor(costs, sp.ORIGINAL, 4, rows=True)
    assert rows == pytest.approx(cols - 2 * costs["launch_ns"] * 1e-3, rel=1e-12, abs=1e-9)
    g_cols = h.level_floor(costs, sp.ORIGINAL, 4, graph=True)
    g_rows = h.level_floor(costs, sp.ORIGINAL, 4, graph=True, rows=True)
    assert g_rows == pytest.approx(g_cols - 2 * costs["graph_node_ns"] * 1e-3, rel=1e-12, abs=1e-9)
    h.set_schedule(sp.ORIGINAL, **SCHEDS[5])  # synchronisation-free: copies by rows stay
    assert h.level_floor(costs, sp.ORIGINAL, 4, rows=True) == h.level_floor(costs, sp.ORIGINAL, 4)
    with pytest.raises(sp.SptrsvError) as ei:
        c, out = sptrsv_mod.LevelCosts(**costs), ctypes.c_double(0)
        h._check(h._L.sptrsv_level_floor(h._h, sp.ORIGINAL, 4, 4, ctypes.byref(c), ctypes.byref(out)))
    assert ei.value.name == "ARG"


def test_rows_autotune(mats):
    """Tuning by rows stores a schedule that both layouts then use, and the
    solve by rows under it matches the oracle; the batched plan is refused."""
    m = mats["stencil3d_tail"]
    h = sp.Handle()
    h.analyze(*dev(m))
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    ms = h.autotune(sp.REWRITTEN, 8, rows=True)
    assert ms > 0
    sched = h.get_schedule(sp.REWRITTEN, 8)
    b_cols = gen.rhs(m, 8)
    bc = torch.from_numpy(b_cols).cuda()
    x_rows = h.solve_rows(bc.t().contiguous(), sp.REWRITTEN)
    x_cols = h.solve(bc, sp.REWRITTEN)
    h.check()
    assert h.get_schedule(sp.REWRITTEN, 8) == sched
    assert torch.equal(x_rows.t(), x_cols)
    assert oracle.relerr(x_cols.cpu().numpy(), oracle.solve(m, b_cols)) <= TOL
    with pytest.raises(sp.SptrsvError) as ei:
        h.autotune(sp.BATCH, 8, rows=True)
    assert ei.value.name == "ARG"


@pytest.mark.parametrize("tc", [1, 2, 4, 8, 16, 3])
@pytest.mark.parametrize("name", ["stencil3d_tail", "window"])
def test_thin_cols(mats, name, tc):
    """Thin runs split over workgroups by columns, in both layouts, with and
    without the rewrite, against the oracle; the two layouts agree bit for bit
    under the same schedule. (The LDS windows are cut for the workgroup's
    columns, so which dependencies a window reads from global memory, and with
    them the rounding, can differ from the unsplit schedule.) A width that
    does not divide nrhs falls back to all columns in one workgroup, bit for
    bit the unsplit result."""
    m = mats[name]
    h = sp.Handle()
    h.analyze(*dev(m))
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    b_cols = gen.rhs(m, 16)
    bc = torch.from_numpy(b_cols).cuda()
    x_ref = oracle.solve(m, b_cols)
    for which in (sp.ORIGINAL, sp.REWRITTEN):
        print(f"thin_cols: {name} tc={tc} which={which}", flush=True)
        h.set_schedule(which, mode=0, thin_rows=256, wg_threads=512)
        ref = h.solve(bc, which)
        h.check()
        h.set_schedule(which, mode=0, thin_rows=256, wg_threads=512, thin_cols=tc)
        assert h.get_schedule(which, 16)["thin_cols"] == tc
        x_cols = h.solve(bc, which)
        x_rows = h.solve_rows(bc.t().contiguous(), which)
        h.check()
        assert torch.equal(x_rows.t(), x_cols)
        assert oracle.relerr(x_cols.cpu().numpy(), x_ref) <= TOL
        if 16 % tc:
            assert torch.equal(x_cols, ref)


@pytest.mark.parametrize("nrhs", [2, 3, 32])
@pytest.mark.parametrize("sched", [dict(mode=1), dict(mode=1, wide_grid=4096), dict(mode=0, thin_rows=8, thin_cols=1),
                                   dict(mode=4, thin_rows=0, wide_threads=256)])
def test_long_rows(sched, nrhs):
    """Wide levels whose rows average at least 16 off-diagonals, with several
    right-hand sides, run with a workgroup per row: against the oracle, both
    layouts bit for bit, plain and rewritten."""
    m = gen.window_random(3000, 11, 96, 48)
    assert (m.nnz - m.n) / m.n >= 16
    h = sp.Handle()
    h.analyze(*dev(m))
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    b_cols = gen.rhs(m, nrhs)
    bc = torch.from_numpy(b_cols).cuda()
    x_ref = oracle.solve(m, b_cols)
    for which in (sp.ORIGINAL, sp.REWRITTEN):
        print(f"long rows: sched={sched} nrhs={nrhs} which={which}", flush=True)
        h.set_schedule(which, **sched)
        x_cols = h.solve(bc, which)
        x_rows = h.solve_rows(bc.t().contiguous(), which)
        h.check()
        assert torch.equal(x_rows.t(), x_cols)
        assert oracle.relerr(x_cols.cpu().numpy(), x_ref) <= TOL
