"""sptrsv_solve_noalloc (work vectors in the library's static work area)
against sptrsv_solve, through the C ABI: the same kernels, so the solutions
must be equal bit for bit, on consecutive calls with a smaller input second,
under every executor; and the host-side refusals (too large, not prepared)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu

sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10

SCHEDULES = {
    "tuned": None,
    "thin": dict(mode=2, thin_rows=0, wg_threads=512),
    "wide": dict(mode=1, wide_threads=256),
    "split": dict(mode=0, thin_rows=64, wg_threads=256),
    "syncfree": dict(mode=3, wide_grid=64),
}


def _setup(m, which, nrhs, sched):
    h = sp.Handle()
    h.analyze(*dev(m))
    if which == sp.REWRITTEN:
        h.rewrite(sp.THIN_ROWS, 32, 4.0)
    if sched is None:
        h.autotune(which, nrhs)
    else:
        h.set_schedule(which, **sched)
    h.prepare(which, nrhs)
    return h


def _pair(h, m, which, nrhs, seed_shift=0):
    b_np = gen.rhs(m, nrhs) + seed_shift
    b = torch.from_numpy(b_np).cuda()
    x_ref = torch.full_like(b, np.nan)
    x_na = torch.full_like(b, np.nan)
    h.solve(b, which, x_ref)
    h.solve(b, which, x_na, noalloc=True)
    h.check()
    return b_np, x_ref.cpu().numpy(), x_na.cpu().numpy()


@pytest.mark.parametrize("sched", list(SCHEDULES))
@pytest.mark.parametrize("which", [sp.ORIGINAL, sp.REWRITTEN])
def test_noalloc_equals_solve_twice_smaller_second(sched, which):
    big = gen.stencil2d_chain(60, 900, 1)        # n = 4,500
    small = gen.window_random(1700, 21, window=40, draws=4)
    print(f"noalloc: sched={sched} which={which} big n={big.n} small n={small.n}", flush=True)
    h1 = _setup(big, which, 3, SCHEDULES[sched])
    b, xr, xn = _pair(h1, big, which, 3)
    assert np.array_equal(xr, xn)
    assert oracle.relerr(xn, oracle.solve(big, b)) <= TOL
    # second call: a smaller matrix and fewer right-hand sides, same work area
    h2 = _setup(small, which, 1, SCHEDULES[sched])
    b2, xr2, xn2 = _pair(h2, small, which, 1, seed_shift=0.25)
    assert np.array_equal(xr2, xn2)
    assert oracle.relerr(xn2, oracle.solve(small, b2)) <= TOL
    # and the first handle again, after the smaller call left its contents behind
    b3, xr3, xn3 = _pair(h1, big, which, 3, seed_shift=-0.5)
    assert np.array_equal(xr3, xn3)
    assert oracle.relerr(xn3, oracle.solve(big, b3)) <= TOL


def test_noalloc_refuses_what_does_not_fit_or_is_not_prepared():
    m = gen.window_random(120_000, 4, window=64, draws=3)
    h = sp.Handle()
    h.analyze(*dev(m))
    b = torch.from_numpy(gen.rhs(m, 2)).cuda()
    x = torch.empty_like(b)
    with pytest.raises(sp.SptrsvError) as e:  # no schedule built for nrhs = 2 yet
        h.solve(b, sp.ORIGINAL, x, noalloc=True)
    assert e.value.name == "STATE"
    h.prepare(sp.ORIGINAL, 2)
    h.solve(b, sp.ORIGINAL, x, noalloc=True)
    h.check()
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, gen.rhs(m, 2))) <= TOL
    nrhs = 4_194_304 // m.n + 1  # one column beyond the work area
    bb = torch.zeros((nrhs, m.n), dtype=torch.float64, device="cuda")
    xx = torch.empty_like(bb)
    h.prepare(sp.ORIGINAL, nrhs)
    with pytest.raises(sp.SptrsvError) as e:
        h.solve(bb, sp.ORIGINAL, xx, noalloc=True)
    assert e.value.name == "ARG"


def test_noalloc_graph_capture_replays():
    """Captured in a hipGraph, replayed three times with eager work between the
    replays; every replay equals the eager allocating solve."""
    m = gen.stencil2d_chain(40, 400, 1)
    h = _setup(m, sp.REWRITTEN, 2, None)
    b_np = gen.rhs(m, 2)
    b = torch.from_numpy(b_np).cuda()
    x_ref = torch.empty_like(b)
    h.solve(b, sp.REWRITTEN, x_ref)
    h.check()
    x = torch.zeros_like(b)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            h.solve(b, sp.REWRITTEN, x, noalloc=True)
    for rep in range(3):
        x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), rep
        y = torch.empty_like(b)
        h.solve(b, sp.REWRITTEN, y)  # eager work between replays
        torch.cuda.synchronize()
    h.check()
