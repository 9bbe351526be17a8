"""GPU parity of solves whose layout transposes run beside the level chain on
the handle's side stream (work vectors of at least 2^22 entries and several
runs): original and rewritten systems, the transposed form (reversed
numbering), eager solves and hipGraph replays, each against the oracle and
bit for bit against the same solve under a schedule with a single run (no
overlap)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10
NRHS = 110  # 39,304 + 600 rows x 110 columns > 2^22 entries per work vector


@pytest.fixture(scope="module")
def mat():
    m = gen.stencil3d_tail(34, 600, 7)
    assert m.n * NRHS >= 1 << 22
    return m


def _solve(h, which, b, sched=None):
    if sched is not None:
        h.set_schedule(which, **sched)
    x = h.solve(b, which)
    h.check()
    return x


SPLIT = [dict(mode=0, thin_rows=64, wg_threads=512, overlap=1),
         dict(mode=4, thin_rows=64, wg_threads=512, wide_threads=256, overlap=1)]


@pytest.mark.parametrize("split", range(len(SPLIT)))
@pytest.mark.parametrize("form", [sp.LOWER, sp.LOWER_TRANS])
@pytest.mark.parametrize("rewrite", [False, True])
def test_overlapped_solve_matches_oracle_and_serial(mat, form, rewrite, split):
    print(f"overlap: form={form} rewrite={rewrite} n={mat.n} nrhs={NRHS}", flush=True)
    b_np = gen.rhs(mat, NRHS)
    xr = oracle.solve(mat, b_np) if form == sp.LOWER else oracle.solve_form(mat, b_np, oracle.LOWER_TRANS)
    h = sp.Handle()
    h.analyze(*dev(mat), form=form)
    which = sp.ORIGINAL
    if rewrite:
        h.rewrite(sp.THIN_ROWS, 32, 4.0)
        which = sp.REWRITTEN
    b = torch.from_numpy(b_np).cuda()
    # split schedule: thin runs and wide launches or dataflow runs -> several runs, overlapped
    x_ovl = _solve(h, which, b, SPLIT[split])
    assert oracle.relerr(x_ovl.cpu().numpy(), xr) <= TOL
    # every level as its own wide launch, same kernels for the wide levels
    x_w = _solve(h, which, b, dict(mode=1))
    assert oracle.relerr(x_w.cpu().numpy(), xr) <= TOL
    # the same split schedule with the transposes in line (profiling disables the overlap)
    h.set_schedule(which, **SPLIT[split])
    h.profile_start()
    x_ser = h.solve(b, which)
    h.profile_stop()
    h.check()
    assert torch.equal(x_ovl, x_ser)


def test_overlapped_graph_replays(mat):
    """Captured in a hipGraph (side-stream work joins the capture), replayed
    three times with eager work in between; every replay equals the eager
    solve."""
    b = torch.from_numpy(gen.rhs(mat, NRHS)).cuda()
    h = sp.Handle()
    h.analyze(*dev(mat))
    h.rewrite(sp.THIN_ROWS, 32, 4.0)
    h.set_schedule(sp.REWRITTEN, mode=0, thin_rows=64, wg_threads=512, overlap=1)
    x_ref = h.solve(b, sp.REWRITTEN)
    h.check()
    x = torch.zeros_like(b)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            h.solve(b, sp.REWRITTEN, x)
    for rep in range(3):
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), rep
        y = h.solve(b, sp.REWRITTEN)
        torch.cuda.synchronize()
        assert torch.equal(y, x_ref)
    with torch.cuda.stream(s):  # the library's own capture needs a stream other than the null stream
        gid = h.graph_create(b, x, sp.REWRITTEN)
        for rep in range(3):
            x.zero_()
            h.graph_launch(gid)
            torch.cuda.synchronize()
            assert torch.equal(x, x_ref), rep
        h.check()
