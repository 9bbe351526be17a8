"""GPU parity of the batched persistent solve: per-matrix levels and solutions
against the oracle, agreement with the per-matrix solves, and replays of a
captured launch (the device work queue resets itself)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10


def _cat(mats):
    rp = np.concatenate([m.row_ptr for m in mats]).astype(np.int32)
    ci = np.concatenate([m.col for m in mats]).astype(np.int32)
    va = np.concatenate([m.val for m in mats])
    return to_dev(rp), to_dev(ci), to_dev(va)


def _rhs_cat(mats, nrhs):
    # matrix i: n_i x nrhs column-major, back to back
    return np.concatenate([gen.rhs(m, nrhs).reshape(-1) for m in mats])


@pytest.fixture(scope="module")
def batch():
    mats, nrhs = gen.config_matrix(3, "small")
    mats = mats + [gen.stencil2d_chain(6, 40, 7), gen.bidiagonal(300, 8)]
    h = sp.Handle()
    h.batch_analyze([m.n for m in mats], *_cat(mats))
    return mats, nrhs, h


def test_batch_levels(batch):
    mats, _, h = batch
    for i, m in enumerate(mats):
        lv = oracle.levels(m)
        lp, lr = h.batch_levels(i)
        assert np.array_equal(lp.cpu().numpy(), lv.level_ptr)
        assert np.array_equal(lr.cpu().numpy(), lv.level_rows)


@pytest.mark.parametrize("nrhs", [1, 16, 5])
def test_batch_solve_parity(batch, nrhs):
    mats, _, h = batch
    b = _rhs_cat(mats, nrhs)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    h.batch_solve(to_dev(b), x, nrhs)
    h.check()
    xs = x.cpu().numpy()
    off = 0
    for m in mats:
        bm = b[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        xm = xs[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        assert oracle.relerr(xm, oracle.solve(m, bm)) <= TOL
        off += m.n


def test_batched_equals_looped_and_single(batch):
    mats, nrhs, h = batch
    b = to_dev(_rhs_cat(mats, nrhs))
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    h.batch_solve(b, x1, nrhs)
    h.batch_solve(b, x2, nrhs, looped=True)
    assert torch.equal(x1, x2)
    # the single-matrix path computes the same rows with the same arithmetic
    m = mats[3]
    off = sum(mm.n for mm in mats[:3])
    hs = sp.Handle()
    hs.analyze(*dev(m))
    bm = b[off * nrhs:(off + m.n) * nrhs].view(nrhs, m.n)
    xs = hs.solve(bm)
    assert torch.equal(xs.reshape(-1), x1[off * nrhs:(off + m.n) * nrhs])


def test_batch_graph_replays(batch):
    mats, nrhs, h = batch
    b = to_dev(_rhs_cat(mats, nrhs))
    x = torch.zeros_like(b)
    h.batch_solve(b, x, nrhs)  # first call prepares work buffers and windows
    ref = x.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            h.batch_solve(b, x, nrhs)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(4):
        x.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, ref)
        _ = (b * 3.0).sum().item()  # eager work between replays


@pytest.mark.parametrize("wg", [256, 1024])
def test_batch_workgroup_sizes(batch, wg):
    mats, nrhs, h = batch
    b = _rhs_cat(mats, nrhs)
    ref = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    h.batch_solve(to_dev(b), ref, nrhs)
    h.set_schedule(sp.BATCH, mode=2, wg_threads=wg)
    assert h.get_schedule(sp.BATCH, nrhs)["wg_threads"] == wg
    x = torch.zeros_like(ref)
    h.batch_solve(to_dev(b), x, nrhs)
    h.check()
    xs = x.cpu().numpy()
    off = 0
    for m in mats:
        xm = xs[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        bm = b[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        assert oracle.relerr(xm, oracle.solve(m, bm)) <= TOL
        off += m.n
    h.set_schedule(sp.BATCH)


def test_batch_autotune(batch):
    mats, nrhs, h = batch
    assert h.autotune(sp.BATCH, nrhs) > 0
    assert h.get_schedule(sp.BATCH, nrhs)["wg_threads"] in (256, 512, 1024)
    b = _rhs_cat(mats, nrhs)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    h.batch_solve(to_dev(b), x, nrhs)
    h.check()
    m = mats[0]
    xm = x[:m.n * nrhs].cpu().numpy().reshape(nrhs, m.n)
    assert oracle.relerr(xm, oracle.solve(m, b[:m.n * nrhs].reshape(nrhs, m.n))) <= TOL
    h.set_schedule(sp.BATCH)


def test_batch_errors():
    h = sp.Handle()
    with pytest.raises(sp.SptrsvError) as ei:
        h._check(h._L.sptrsv_batch_solve(h._h, 1, None, None, None))
    assert ei.value.name in ("STATE", "ARG")


@pytest.mark.parametrize("nrhs", [16, 1])
@pytest.mark.parametrize("wide_first", [False, True])
def test_batch_with_levels_too_wide_for_a_window(nrhs, wide_first):
    """A uniform random lower-triangular matrix (n = 50,000, about 6 nonzeros
    per row, columns anywhere before the row) has levels of thousands of rows,
    too wide for one workgroup's LDS window at 16 right-hand sides: it is
    solved level by level beside the persistent launch, in the same call, and
    every matrix still matches the oracle; the looped per-matrix solve gives
    the same bits."""
    wide = gen.window_random(50_000, 17, window=50_000, draws=6)
    widths = np.diff(oracle.levels(wide).level_ptr)
    assert widths.max() > 2000
    small = [gen.window_random(3000 + 500 * i, 40 + i) for i in range(5)]
    mats = [wide] + small if wide_first else small[:3] + [wide] + small[3:]
    h = sp.Handle()
    h.batch_analyze([m.n for m in mats], *_cat(mats))
    b = _rhs_cat(mats, nrhs)
    bd = to_dev(b)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    h.batch_solve(bd, x, nrhs)
    h.check()
    xs = x.cpu().numpy()
    off = 0
    for m in mats:
        bm = b[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        xm = xs[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        assert oracle.relerr(xm, oracle.solve(m, bm)) <= TOL
        off += m.n
    x2 = torch.zeros_like(x)
    h.batch_solve(bd, x2, nrhs, looped=True)
    h.check()
    assert torch.equal(x, x2)
