"""Pins for the FP64 MLP oracle (finite differences, torch autograd and
torch's Adam in float64) and for the per-level policy features (brute force)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import mlp


def _batch(seed, B=37):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(B, mlp.F_IN))
    y = (rng.random(B) < 0.4).astype(np.float64)
    th = mlp.init(seed) + rng.normal(scale=0.05, size=mlp.NPARAM)  # nonzero biases
    return th, f, y


def test_param_count():
    assert mlp.F_IN == oracle.NFEAT == 20
    assert mlp.NPARAM == 20 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5569


def test_gradient_finite_differences():
    th, f, y = _batch(1)
    g, _ = mlp.backward(th, f, y)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, f, y) - mlp.loss(th - e, f, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def test_against_torch_autograd():
    th, f, y = _batch(3)
    g, lval = mlp.backward(th, f, y)
    p = mlp.unpack(th)
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    x = torch.tensor(f)
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    z = h2 @ t["W3"] + t["b3"]
    L = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(y))
    L.backward()
    gt = np.concatenate([t[k].grad.numpy().reshape(-1) for k, _ in mlp.SIZES])
    assert abs(L.item() - lval) < 1e-13
    np.testing.assert_allclose(g, gt, rtol=1e-11, atol=1e-15)
    prob, _ = mlp.forward(th, f)
    np.testing.assert_allclose(prob, torch.sigmoid(z).detach().numpy(), rtol=1e-14)


def test_adam_against_torch():
    th, f, y = _batch(4)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    tt = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g, _ = mlp.backward(th, f, y)
        th, m, v = mlp.adam(th, g, m, v, step, 3e-3)
        opt.zero_grad()
        tt.grad = torch.tensor(mlp.backward(tt.detach().numpy(), f, y)[0])
        opt.step()
    np.testing.assert_allclose(th, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_brute_force():
    m = gen.window_random(300, 8, window=6, draws=3)
    lv = oracle.levels(m)
    F = oracle.level_features(m, lv)
    c = oracle.level_costs(m, lv)
    assert F.shape == (lv.nlev, 20)
    nnz = np.diff(m.row_ptr)
    for l in range(lv.nlev):
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        R = len(rows)
        assert F[l, 0] == pytest.approx(np.log1p(R))
        assert F[l, 1] == pytest.approx(np.log1p(nnz[rows].sum()))
        assert F[l, 2] == pytest.approx(np.log1p(np.sum(2 * nnz[rows] - 1)))
        assert F[l, 3] == pytest.approx(np.sum(2 * nnz[rows] - 1) / (c.total / lv.nlev))
        off = nnz[rows] - 1
        bins = [off == 0, off == 1, off == 2, (off >= 3) & (off <= 4), (off >= 5) & (off <= 8), off >= 9]
        for bi, bm in enumerate(bins):
            assert F[l, 6 + bi] == pytest.approx(bm.mean())
        assert F[l, 14] == pytest.approx(l / lv.nlev)
    _check_size_features(m, lv, F)
    # features 12, 13: a single-level move toward the level before; compare with
    # the oracle's own rewrite restricted to that one level (mask with one source)
    for l in [1, 2, lv.nlev // 2, lv.nlev - 1]:
        mask = np.zeros(lv.nlev, np.uint8)
        mask[l] = 1
        rw = oracle.rewrite(m, oracle.THIN_ROWS, 1e9, 0.0, 0, mask, lv)
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        assert np.all(rw.target[rows] == l - 1)
        lp = np.diff(rw.lp_ptr)[rows].sum()
        tn = np.diff(rw.t_ptr)[rows].sum()
        assert F[l, 12] == pytest.approx(lp / nnz[rows].sum())
        assert F[l, 13] == pytest.approx(np.log1p(tn))


def _check_size_features(m, lv, F):
    """Features 4, 5 and 15 by direct count over the rows of each level: rows
    over 32, mean nnz per row (diagonal included), and log1p of the number of
    rows of the level before (0 for level 0)."""
    nnz = np.diff(m.row_ptr)
    sizes = np.diff(lv.level_ptr)
    for l in range(lv.nlev):
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        assert F[l, 4] == pytest.approx(len(rows) / 32.0)
        assert F[l, 5] == pytest.approx(nnz[rows].sum() / len(rows))
        assert F[l, 15] == pytest.approx(np.log1p(sizes[l - 1]) if l > 0 else 0.0)


def _size_feature_case():
    """A matrix whose consecutive levels differ in size and in mean row
    length, so that reading the wrong level or the wrong count shows."""
    return gen.window_random(400, 11, window=9, draws=4)


@pytest.mark.parametrize("old,new", [("f[4] = R / 32.0;", "f[4] = R / 31.0;"),
                                     ("f[5] = R > 0.0 ? (double)nzl[l] / R : 0.0;",
                                      "f[5] = R > 0.0 ? (double)(nzl[l] - rows[l]) / R : 0.0;"),
                                     ("f[15] = l > 0 ? log1p((double)rows[l - 1]) : 0.0;",
                                      "f[15] = l > 0 ? log1p((double)rows[l]) : 0.0;")])
def test_planted_size_feature_errors_are_caught(tmp_path, old, new):
    """A planted mistake in feature 4, 5 or 15 (a wrong divisor, the
    off-diagonal count in place of nnz, the current level's rows in place of
    the previous level's) fails the direct count."""
    from tests.test_oracle_rewrite import _with_planted_oracle
    m = _size_feature_case()

    def check():
        lv = oracle.levels(m)
        with pytest.raises(AssertionError):
            _check_size_features(m, lv, oracle.level_features(m, lv))

    _with_planted_oracle(tmp_path, old, new, check)


def test_size_features_direct_count():
    m = _size_feature_case()
    lv = oracle.levels(m)
    _check_size_features(m, lv, oracle.level_features(m, lv))


def _heights_by_dependents(m):
    """Longest path from each row to a row nothing depends on, by memoised
    recursion over the dependents (the other direction from the oracle's
    sweep over dependencies)."""
    dependents = [[] for _ in range(m.n)]
    for r in range(m.n):
        for p in range(m.row_ptr[r], m.row_ptr[r + 1] - 1):
            dependents[int(m.col[p])].append(r)
    h = [None] * m.n
    for r in range(m.n - 1, -1, -1):  # dependents have larger indices
        h[r] = 1 + max((h[d] for d in dependents[r]), default=-1)
    return np.array(h)


def _moved_rows(m, lv, l):
    """Off-diagonal columns of each row of level l after the distance-1 move
    (the oracle's rewrite with a one-level mask), or the rows as they are for
    level 0."""
    rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
    if l == 0:
        return [m.col[m.row_ptr[r]:m.row_ptr[r + 1] - 1] for r in rows]
    mask = np.zeros(lv.nlev, np.uint8)
    mask[l] = 1
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 1e9, 0.0, 0, mask, lv)
    out = []
    for r in rows:
        c = rw.lp.col[rw.lp.row_ptr[r]:rw.lp.row_ptr[r + 1]]
        out.append(c[c != r])
    return out


@pytest.mark.parametrize("case", ["window", "powerlaw"])
def test_row_constraint_features_brute_force(case):
    """Features 16..19 (the Sec. III.A row constraints on the distance-1 move)
    against a direct count over the moved rows."""
    m = gen.window_random(300, 8, window=6, draws=3) if case == "window" else gen.powerlaw(3000, seed=5, w_loc=2048, nseg=2, seglen=50)
    lv = oracle.levels(m)
    F = oracle.level_features(m, lv)
    h = _heights_by_dependents(m)
    for l in range(lv.nlev):
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        cols = _moved_rows(m, lv, l)
        span = np.array([int(c.max()) - int(c.min()) if len(c) else 0 for c in cols])
        assert F[l, 16] == pytest.approx(np.mean([len(c) < 4 for c in cols]))
        assert F[l, 17] == pytest.approx(np.mean(l + h[rows] == lv.nlev - 1))
        assert F[l, 18] == pytest.approx(np.log1p(span.mean()))
        assert F[l, 19] == pytest.approx(np.mean(span < 1024))


def test_critical_path_feature_two_chains():
    """Two independent chains of lengths 6 and 3 (rows 0..5 and 6..8): the
    longest path is the long chain, so its rows are critical and the short
    chain's are not; levels 0..2 hold one row of each, levels 3..5 only the
    long chain's."""
    import gen as G
    rp, ci, va = [0], [], []
    for r in range(9):
        if r not in (0, 6):
            ci.append(r - 1)
            va.append(-0.5)
        ci.append(r)
        va.append(2.0)
        rp.append(len(ci))
    m = G.Csr(9, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))
    lv = oracle.levels(m)
    F = oracle.level_features(m, lv)
    assert lv.nlev == 6
    np.testing.assert_allclose(F[:, 17], [0.5, 0.5, 0.5, 1.0, 1.0, 1.0])


@pytest.mark.parametrize("old,new", [("n_alpha += na < 4;", "n_alpha += na <= 4;"),
                                     ("n_local += span < 1024;", "n_local += span <= 1024;"),
                                     ("n_crit += lev[r] + height[r] == nlev - 1;", "n_crit += lev[r] + height[r] >= nlev - 2;")])
def test_planted_feature_errors_are_caught(tmp_path, old, new):
    """Each row-constraint feature with a planted boundary error fails its
    brute-force pin on a matrix where that boundary occurs (seed 8: a moved
    row spans exactly 1024 columns, five keep exactly 4 dependencies, and 56
    rows lie one level short of a longest path)."""
    from tests.test_oracle_rewrite import _with_planted_oracle
    m = gen.powerlaw(3000, seed=8, w_loc=2048, nseg=2, seglen=50)

    def check():
        with pytest.raises(AssertionError):
            _brute(m)

    _with_planted_oracle(tmp_path, old, new, check)


def _brute(m):
    """Features 16..19 of m against the direct count (the pin above)."""
    lv = oracle.levels(m)
    F = oracle.level_features(m, lv)
    h = _heights_by_dependents(m)
    for l in range(lv.nlev):
        rows = lv.level_rows[lv.level_ptr[l]:lv.level_ptr[l + 1]]
        cols = _moved_rows(m, lv, l)
        span = np.array([int(c.max()) - int(c.min()) if len(c) else 0 for c in cols])
        assert F[l, 16] == pytest.approx(np.mean([len(c) < 4 for c in cols]))
        assert F[l, 17] == pytest.approx(np.mean(l + h[rows] == lv.nlev - 1))
        assert F[l, 18] == pytest.approx(np.log1p(span.mean()))
        assert F[l, 19] == pytest.approx(np.mean(span < 1024))
