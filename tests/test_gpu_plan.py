"""Plan files through the C ABI: analyse, rewrite and tune in one handle, save,
load into a fresh handle, and compare levels, L', T, targets, schedules and x
bit for bit (no analysis, rewrite or tuning in the loading handle); files that
are truncated, altered, of another kind or missing are refused with ERR_ARG
and leave the loading handle as it was."""
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10


def _built(m, nrhs, form=None, rewrite=True):
    h = sp.Handle()
    if form is None:
        h.analyze(*dev(m))
    else:
        h.analyze(*dev(m), form=form)
    which = sp.ORIGINAL
    if rewrite:
        h.rewrite(sp.THIN_ROWS, 32, 4.0)
        which = sp.REWRITTEN
    h.autotune(which, nrhs)
    h.autotune(sp.ORIGINAL, nrhs)
    return h, which


@pytest.mark.parametrize("case,nrhs,form", [("stencil_chain", 1, None), ("window", 3, None),
                                            ("stencil3d", 4, None), ("stencil_chain_T", 2, "lower_trans")])
def test_plan_roundtrip_bit_exact(tmp_path, case, nrhs, form):
    m = {"stencil_chain": lambda: gen.stencil2d_chain(40, 500, 1), "window": lambda: gen.window_random(9000, 3, 50, 6),
         "stencil3d": lambda: gen.stencil3d_tail(18, 200, 4),
         "stencil_chain_T": lambda: gen.stencil2d_chain(30, 300, 2)}[case]()
    f = {None: None, "lower_trans": sp.LOWER_TRANS}[form]
    print(f"plan: case={case} n={m.n} nrhs={nrhs}", flush=True)
    h1, which = _built(m, nrhs, f)
    path = str(tmp_path / "p.plan")
    h1.plan_save(path)
    h2 = sp.Handle()
    info = h2.plan_load(path)
    assert info["n"] == m.n and info["has_rewrite"] and info["nlev"] == h1.nlev
    assert h2.rstats == h1.rstats
    for w in (sp.ORIGINAL, sp.REWRITTEN):
        a, b = h1.levels(w), h2.levels(w)
        for t1, t2 in zip(a, b):
            assert torch.equal(t1, t2)
        assert h1.get_schedule(w, nrhs) == h2.get_schedule(w, nrhs)
    g1, g2 = h1.rewritten(), h2.rewritten()
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k
    assert torch.equal(h1.targets(), h2.targets())
    b = torch.from_numpy(gen.rhs(m, nrhs)).cuda()
    for w in (sp.ORIGINAL, sp.REWRITTEN):
        x1 = h1.solve(b, w)
        x2 = h2.solve(b, w)
        h1.check()
        h2.check()
        assert torch.equal(x1, x2)
    xr = oracle.solve(m, b.cpu().numpy()) if f is None else oracle.solve_form(m, b.cpu().numpy(), oracle.LOWER_TRANS)
    assert oracle.relerr(x2.cpu().numpy(), xr) <= TOL
    # the residual check uses the stored matrix
    assert max(h2.residual(b, x2)) == max(h1.residual(b, x1))


def test_plan_without_rewrite(tmp_path):
    m = gen.window_random(3000, 8, 30, 5)
    h1, _ = _built(m, 2, rewrite=False)
    path = str(tmp_path / "q.plan")
    h1.plan_save(path)
    h2 = sp.Handle()
    info = h2.plan_load(path)
    assert not info["has_rewrite"]
    b = torch.from_numpy(gen.rhs(m, 2)).cuda()
    assert torch.equal(h1.solve(b), h2.solve(b))
    with pytest.raises(sp.SptrsvError) as e:
        h2.solve(b, sp.REWRITTEN)
    assert e.value.name == "STATE"


def test_bad_plan_files_are_refused(tmp_path):
    m = gen.stencil2d_chain(20, 100, 3)
    h1, _ = _built(m, 1)
    path = str(tmp_path / "good.plan")
    h1.plan_save(path)
    raw = open(path, "rb").read()
    other = gen.window_random(500, 4, 20, 3)
    h2 = sp.Handle()
    h2.analyze(*dev(other))  # what the handle holds must survive a refused load
    b2 = torch.from_numpy(gen.rhs(other, 1)).cuda()
    x_before = h2.solve(b2)
    bad = {
        "truncated": raw[: len(raw) // 2],
        "tail_cut": raw[:-3],
        "one_bit": raw[:200] + bytes([raw[200] ^ 0x10]) + raw[201:],
        "not_a_plan": b"hello world" * 10,
        "empty": b"",
        "version": raw[:8] + (99).to_bytes(4, "little") + raw[12:],
    }
    for name, data in bad.items():
        p = str(tmp_path / f"{name}.plan")
        with open(p, "wb") as f:
            f.write(data)
        with pytest.raises(sp.SptrsvError) as e:
            h2.plan_load(p)
        assert e.value.name == "ARG", name
    with pytest.raises(sp.SptrsvError) as e:
        h2.plan_load(str(tmp_path / "missing.plan"))
    assert e.value.name == "ARG"
    assert torch.equal(h2.solve(b2), x_before)
    assert os.path.getsize(path) == len(raw)
