"""The input recipes realise what they state: the power-law matrix holds
d_i = min(Poisson(8), i) distinct off-diagonals in row i (mean 8 per row at
the full 4M-row size), and the redraws over the columns a row lacks never
return a held column."""
import numpy as np

import gen
from gen import matrices as gm


def _drawn_degrees(n, seed, mean_deg=8.0):
    """The per-row counts the recipe draws: its generator's first two draws
    are the weight permutation and the Poisson counts."""
    rng = np.random.default_rng(seed)
    rng.permutation(n)
    return np.minimum(rng.poisson(mean_deg, n), np.arange(n))


def test_powerlaw_rows_hold_their_drawn_count():
    n, seed = 60_000, 2
    m = gen.powerlaw(n, seed, w_loc=512, nseg=4, seglen=60)
    off = np.diff(m.row_ptr) - 1
    np.testing.assert_array_equal(off, _drawn_degrees(n, seed))
    for r in range(n):  # strictly ascending, lower, diagonal last
        c = m.col[m.row_ptr[r]:m.row_ptr[r + 1]]
        assert c[-1] == r and np.all(np.diff(c) > 0)


def test_powerlaw_full_size_mean_degree():
    """The benchmark's power-law matrix: within 2 % of 8 off-diagonals per row."""
    m, _ = gen.config_matrix(2)
    mean = (m.nnz - m.n) / m.n
    assert m.n == 4_000_000
    assert abs(mean - 8.0) <= 0.02 * 8.0, mean


def test_draw_excluding_never_returns_a_held_column():
    rng = np.random.default_rng(7)
    n = 50
    w = (rng.permutation(n) + 1.0) ** -1.2
    cumw = np.cumsum(w)
    rows = np.array([5, 9, 30, 49])
    held = {5: [0, 1, 2], 9: [3, 8], 30: list(range(0, 30, 2)), 49: [int(np.argmax(w[:49]))]}
    keys = np.sort(np.array([r * n + c for r in rows for c in held[int(r)]], np.int64))
    need = np.array([2, 7, 15, 10])
    out = gm._draw_excluding(rng, cumw, keys, rows, need, n)
    for r, k in zip(rows, need):
        cols = out[out // n == r] % n
        assert len(cols) == k and len(set(cols.tolist())) == k
        assert np.all(cols < r) and not set(cols.tolist()) & set(held[int(r)])
    # rows 5 and 30 lack exactly the columns drawn: all of them are taken
    assert sorted((out[out // n == 5] % n).tolist()) == [3, 4]
    assert sorted((out[out // n == 30] % n).tolist()) == list(range(1, 30, 2))


def test_draw_excluding_follows_the_weights():
    """Drawing one column from [0, r) minus a held set many times gives the
    weights renormalised over the free columns."""
    rng = np.random.default_rng(3)
    n, r = 40, 12
    w = (rng.permutation(n) + 1.0) ** -1.2
    cumw = np.cumsum(w)
    top = int(np.argmax(w[:r]))
    held = [top, 7 if top != 7 else 6]
    keys = np.sort(np.array([r * n + c for c in held], np.int64))
    reps = 20_000
    out = gm._draw_excluding(rng, cumw, keys, np.full(reps, r), np.ones(reps, np.int64), n) % n
    freq = np.bincount(out, minlength=r)[:r] / reps
    p = w[:r].copy()
    p[held] = 0.0
    p /= p.sum()
    assert freq[held].sum() == 0
    np.testing.assert_allclose(freq, p, atol=0.015)
