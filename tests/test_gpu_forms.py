"""GPU parity of the other triangular forms a preconditioner application needs
(U x = b, L^T x = b, U^T x = b) against the oracle's backward and transposed
substitutions, through the C ABI: x, levels of the lower form the handle
keeps, rewriting of that form, residuals, errors, and z = L^-T L^-1 r."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10
FORMS = {"upper": sp.UPPER, "lower_trans": sp.LOWER_TRANS, "upper_trans": sp.UPPER_TRANS}


def _mats():
    yield "bidiag", gen.bidiagonal(700, 2)
    yield "cfg0", gen.config_matrix(0)[0]
    yield "cfg1_small", gen.config_matrix(1, "small")[0]
    yield "cfg4_small", gen.config_matrix(4, "small")[0]
    yield "window_ragged", gen.window_random(3001, 9, window=200, draws=7)


MATS = list(_mats())


def _input(m, form):
    """The CSR the caller hands in for this form (upper forms get L^T)."""
    return gen.transpose(m) if form in (sp.UPPER, sp.UPPER_TRANS) else m


def _reverse(a):
    """J A J of a CSR, written out in the test (rows and columns reversed)."""
    n, nnz = a.n, int(a.row_ptr[-1])
    return gen.Csr(n, (nnz - a.row_ptr[::-1]).astype(np.int32), (n - 1 - a.col[::-1]).astype(np.int32),
                   a.val[::-1].copy(), a.name + "_rev")


def _lower_form(m, form):
    """The lower-triangular system the handle keeps for each form."""
    a = _input(m, form)
    if form == sp.UPPER:
        return _reverse(a)
    if form == sp.LOWER_TRANS:
        return _reverse(gen.transpose(a))
    return gen.transpose(a)  # UPPER_TRANS: U^T


@pytest.mark.parametrize("name", [n for n, _ in MATS])
@pytest.mark.parametrize("fname", list(FORMS))
@pytest.mark.parametrize("nrhs", [1, 5])
def test_form_solve_parity(name, fname, nrhs):
    m = dict(MATS)[name]
    form = FORMS[fname]
    a = _input(m, form)
    h = sp.Handle()
    nlev = h.analyze(*dev(a), form=form)
    lv = oracle.levels(_lower_form(m, form))
    assert nlev == lv.nlev
    lp, lr, _ = (t.cpu().numpy() for t in h.levels())
    assert np.array_equal(lp, lv.level_ptr) and np.array_equal(lr, lv.level_rows)
    b = gen.rhs(m, nrhs)
    xr = oracle.solve_form(a, b, form)
    # strided b and x
    bd = torch.zeros((nrhs, m.n + 11), dtype=torch.float64, device="cuda")
    bd[:, :m.n] = to_dev(b.reshape(nrhs, m.n))
    xd = torch.full((nrhs, m.n + 3), float("nan"), dtype=torch.float64, device="cuda")
    bb, xx = (bd[:, :m.n], xd[:, :m.n]) if nrhs > 1 else (bd[0, :m.n], xd[0, :m.n])
    h.solve(bb, sp.ORIGINAL, xx)
    h.check()
    assert oracle.relerr(xd[:, :m.n].cpu().numpy(), xr.reshape(nrhs, m.n)) <= TOL
    assert torch.isnan(xd[:, m.n:]).all()
    res = h.residual(bb, xx)
    assert max(res) <= 1e-12 * (1.0 + float(np.abs(xr).max()))


@pytest.mark.parametrize("workers", [1, 2])
@pytest.mark.parametrize("fname", list(FORMS))
@pytest.mark.parametrize("name", ["cfg1_small", "window_ragged"])
def test_form_rewrite_parity(fname, name, workers):
    # the rewrite runs on the lower form the handle keeps (for U and L^T: the
    # reverse row order), bit for bit with the oracle on that form, with the
    # scan from one end or from both; x in the caller's numbering
    m = dict(MATS)[name]
    form = FORMS[fname]
    a = _input(m, form)
    low = _lower_form(m, form)
    h = sp.Handle()
    h.analyze(*dev(a), form=form)
    st = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0, scan_workers=workers)
    lv = oracle.levels(low)
    rw = oracle.rewrite(low, oracle.THIN_ROWS, 32.0, 4.0, 0, None, lv, both_ends=workers > 1)
    assert st["rows_rewritten"] == rw.rows_rewritten and st["nlev_after"] == oracle.levels(rw.lp).nlev
    g = {k: v.cpu().numpy() for k, v in h.rewritten().items()}
    for k in ("lp_ptr", "lp_col", "lp_val", "t_ptr", "t_col", "t_val"):
        assert np.array_equal(g[k], getattr(rw, k)), k
    assert np.array_equal(h.targets().cpu().numpy(), rw.target)
    b = gen.rhs(m, 3)
    x = h.solve(to_dev(b), sp.REWRITTEN)
    h.check()
    assert oracle.relerr(x.cpu().numpy(), oracle.solve_form(a, b, form)) <= TOL
    h.autotune(sp.REWRITTEN, 3)
    x2 = h.solve(to_dev(b), sp.REWRITTEN)
    assert oracle.relerr(x2.cpu().numpy(), oracle.solve_form(a, b, form)) <= TOL


def test_preconditioner_application():
    # z = L^-T L^-1 r (an incomplete-Cholesky-style application) with two
    # handles, once with L^T given implicitly and once as an explicit U
    m = gen.config_matrix(4, "small")[0]
    r = gen.rhs(m, 4)
    zr = oracle.solve_form(m, oracle.solve(m, r), oracle.LOWER_TRANS)
    hl, ht, hu = sp.Handle(), sp.Handle(), sp.Handle()
    hl.analyze(*dev(m))
    ht.analyze(*dev(m), form=sp.LOWER_TRANS)
    hu.analyze(*dev(gen.transpose(m)), form=sp.UPPER)
    y = hl.solve(to_dev(r))
    z1 = ht.solve(y)
    z2 = hu.solve(y)
    for h in (hl, ht, hu):
        h.check()
    assert oracle.relerr(z1.cpu().numpy(), zr) <= TOL
    assert oracle.relerr(z2.cpu().numpy(), zr) <= TOL


def test_form_errors():
    m = gen.window_random(300, 1, window=8, draws=3)
    h = sp.Handle()
    with pytest.raises(sp.SptrsvError) as ei:  # a lower matrix is not upper-triangular
        h.analyze(*dev(m), form=sp.UPPER)
    assert ei.value.name == "NOT_LOWER"
    with pytest.raises(sp.SptrsvError) as ei:
        h.analyze(*dev(gen.transpose(m)), form=sp.LOWER_TRANS)
    assert ei.value.name == "NOT_LOWER"
    with pytest.raises(sp.SptrsvError) as ei:
        h.analyze(*dev(m), form=7)
    assert ei.value.name == "ARG"
    # empty and single-row systems
    for f in FORMS.values():
        h = sp.Handle()
        e = gen.diagonal(1, 2)
        assert h.analyze(*dev(e), form=f) == 1
        b = gen.rhs(e, 1)
        assert oracle.relerr(h.solve(to_dev(b[0])).cpu().numpy(), oracle.solve_form(e, b, f)) <= TOL


@pytest.mark.parametrize("fname", list(FORMS))
def test_form_level_features(fname):
    # the learned policy's features describe the lower form the handle keeps
    m = dict(MATS)["cfg1_small"]
    form = FORMS[fname]
    h = sp.Handle()
    h.analyze(*dev(_input(m, form)), form=form)
    f = h.level_features().cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(f, oracle.level_features(_lower_form(m, form)), rtol=2e-6, atol=1e-6)
