"""Seeded generators for sparse lower-triangular CSR systems.

Every generator follows the same conventions:

* CSR with int32 ``row_ptr``/``col`` and float64 ``val``; columns strictly
  ascending in each row, the diagonal stored last (the layout the paper's
  serial algorithm assumes, Sec. II.A, Algorithm 1).
* Off-diagonal values are drawn U(-1, 1) in CSR order after the sparsity
  pattern is fixed; the diagonal is ``1 + sum(|off-diagonals|)`` so every
  matrix is strictly diagonally dominant by rows.
* ``rhs(m, nrhs)`` draws U(-1, 1) right-hand sides from the same generator,
  continuing after the matrix draws; it is column-major, shape (nrhs, n).

The recipes stand in for the paper's SuiteSparse workloads (Sec. IV): fat,
parallel regions next to long runs of thin, near-serial levels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Csr", "window_random", "stencil2d_chain", "stencil3d_tail", "powerlaw",
    "batch_window", "policy_training_matrix", "rhs", "from_dense_lower", "bidiagonal", "diagonal",
    "config_matrix",
]


@dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    name: str = ""
    rng_state: dict | None = field(default=None, repr=False)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _assemble(n, rows, cols, rng, name):
    """Build the CSR from sorted, de-duplicated off-diagonal (rows, cols)
    pairs, then draw the values with ``rng``."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    noff = np.bincount(rows, minlength=n).astype(np.int64) if rows.size else np.zeros(n, np.int64)
    counts = noff + 1
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("matrix too large for int32 indices")
    nnz = int(row_ptr[-1])
    offv = rng.uniform(-1.0, 1.0, size=rows.size)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    # position of each off-diagonal: row start + rank within its row
    off_start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(noff, out=off_start[1:])
    rank = np.arange(rows.size, dtype=np.int64) - off_start[rows]
    pos = row_ptr[rows] + rank
    col[pos] = cols
    val[pos] = offv
    dpos = row_ptr[1:] - 1
    col[dpos] = np.arange(n, dtype=np.int32)
    absum = np.zeros(n, dtype=np.float64)
    if rows.size:
        np.add.at(absum, rows, np.abs(offv)) if rows.size < 4096 else None
        if rows.size >= 4096:
            absum = np.bincount(rows, weights=np.abs(offv), minlength=n)
    val[dpos] = 1.0 + absum
    return Csr(n, row_ptr.astype(np.int32), col, val, name, rng.bit_generator.state)


def _unique_pairs(n, rows, cols):
    key = np.unique(np.asarray(rows, np.int64) * n + np.asarray(cols, np.int64))
    return key // n, key % n


def window_random(n: int, seed: int, window: int = 64, draws: int = 5) -> Csr:
    """Row i draws ``draws`` columns uniformly, with replacement, from
    [max(0, i-window), i-1] and keeps the distinct ones ("up to 5")."""
    rng = np.random.default_rng(seed)
    if n > 1:
        i = np.arange(1, n, dtype=np.int64)
        lo = np.maximum(0, i - window)
        c = rng.integers(lo[:, None], i[:, None], size=(n - 1, draws))
        r = np.repeat(i, draws)
        rows, cols = _unique_pairs(n, r, c.reshape(-1))
    else:
        rows = cols = np.zeros(0, np.int64)
    return _assemble(n, rows, cols, rng, f"window{window}_n{n}_s{seed}")


def _chain_pairs(rng, first: int, count: int):
    """Chain rows q in [first, first+count): q-1 plus 2 distinct columns
    uniform in [0, q-2] (fewer when q-1 < 2)."""
    q = np.arange(first, first + count, dtype=np.int64)
    if count == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if first < 3:
        raise ValueError("chain must start at row >= 3")
    m = q - 1  # number of candidates in [0, q-2]
    a = rng.integers(0, m)
    c = rng.integers(0, m - 1)
    c = c + (c >= a)
    rows = np.concatenate([q, q, q])
    cols = np.concatenate([a, c, q - 1])
    return rows, cols


def stencil2d_chain(k: int = 1000, chain: int = 20000, seed: int = 1) -> Csr:
    """Lower triangle of the k x k 5-point stencil in natural order
    (p = k*i + j depends on p-k and p-1), then ``chain`` near-serial rows."""
    rng = np.random.default_rng(seed)
    n0 = k * k
    p = np.arange(n0, dtype=np.int64)
    i, j = p // k, p % k
    r_up, c_up = p[i > 0], p[i > 0] - k
    r_lf, c_lf = p[j > 0], p[j > 0] - 1
    cr, cc = _chain_pairs(rng, n0, chain)
    rows = np.concatenate([r_up, r_lf, cr])
    cols = np.concatenate([c_up, c_lf, cc])
    rows, cols = _unique_pairs(n0 + chain, rows, cols)
    return _assemble(n0 + chain, rows, cols, rng, f"stencil2d_k{k}_chain{chain}_s{seed}")


def stencil3d_tail(k: int = 200, tail: int = 5000, seed: int = 4) -> Csr:
    """Lower triangle of the k^3 7-point stencil, p = (k*i + j)*k + l, with
    dependencies p-k^2, p-k, p-1; then a ``tail`` of chain rows."""
    rng = np.random.default_rng(seed)
    n0 = k * k * k
    p = np.arange(n0, dtype=np.int64)
    i, j, l = p // (k * k), (p // k) % k, p % k
    parts_r = [p[i > 0], p[j > 0], p[l > 0]]
    parts_c = [p[i > 0] - k * k, p[j > 0] - k, p[l > 0] - 1]
    cr, cc = _chain_pairs(rng, n0, tail)
    rows = np.concatenate(parts_r + [cr])
    cols = np.concatenate(parts_c + [cc])
    rows, cols = _unique_pairs(n0 + tail, rows, cols)
    return _assemble(n0 + tail, rows, cols, rng, f"stencil3d_k{k}_tail{tail}_s{seed}")


def powerlaw(n: int = 4_000_000, seed: int = 2, mean_deg: float = 8.0, w_loc: int = 4096,
             nseg: int = 8, seglen: int = 250, alpha: float = 1.2) -> Csr:
    """Power-law in-degree: column weights pi(j)^-alpha for a random
    permutation pi. Row i takes d_i = min(Poisson(mean_deg), i) distinct
    off-diagonals: one local column uniform in [i-w_loc, i-1], the rest drawn
    by inverse CDF over the weights restricted to [0, i). A draw that repeats
    a column the row already holds is drawn again from the same weights, so
    every row ends with d_i distinct columns and the realised mean is
    mean_deg (the hub columns make repeats frequent: without the redraws
    about a quarter of the draws would be lost). Redraws run in rounds over
    all rows still short; the few rows left after that (their weights are
    dominated by hub columns they already hold) draw from the weights of the
    columns they lack, one column at a time. ``nseg`` segments of ``seglen``
    rows use a local window of 1, which makes them near-serial."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.float64) + 1.0
    w = perm ** (-alpha)
    cumw = np.cumsum(w)
    deg = np.minimum(rng.poisson(mean_deg, n), np.arange(n))
    wl = np.full(n, w_loc, dtype=np.int64)
    for s in range(nseg):
        st = ((s + 1) * n) // (nseg + 1)
        wl[st:st + seglen] = 1
    has = np.nonzero(deg >= 1)[0].astype(np.int64)
    lo = np.maximum(0, has - wl[has])
    loc = rng.integers(lo, has)
    extra = (deg[has] - 1).astype(np.int64)
    er = np.repeat(has, extra)
    u = rng.random(er.size) * cumw[er - 1]
    ec = np.minimum(_inv_cdf(cumw, u), er - 1)
    keys = np.unique(np.concatenate([has * n + loc, er * n + ec]))
    got = np.bincount(keys // n, minlength=n)
    added = np.zeros(0, np.int64)  # accepted redraws, sorted
    for _ in range(40):
        short = np.nonzero(got < deg)[0].astype(np.int64)
        if short.size <= 20_000:
            break
        rr = np.repeat(short, (deg[short] - got[short]).astype(np.int64))
        u = rng.random(rr.size) * cumw[rr - 1]
        cc = np.minimum(_inv_cdf(cumw, u), rr - 1)
        # distinct within the round; a row drew exactly its shortfall, so
        # every fresh key fits
        cand = np.unique(rr * n + cc)
        new = cand[~_contains(keys, cand) & ~_contains(added, cand)]
        added = np.sort(np.concatenate([added, new]))
        got += np.bincount(new // n, minlength=n)
    keys = np.sort(np.concatenate([keys, added]))
    short = np.nonzero(got < deg)[0].astype(np.int64)
    if short.size:
        keys = np.sort(np.concatenate([keys, _draw_excluding(rng, cumw, keys, short, deg[short] - got[short], n)]))
    return _assemble(n, keys // n, keys % n, rng, f"powerlaw_n{n}_s{seed}_w{w_loc}_g{nseg}")


def _inv_cdf(cumw, u):
    """Index of the first cumulative weight above each u (inverse CDF); the
    queries are searched in sorted order, which keeps the search cache-local,
    and the results are put back in the order of u."""
    order = np.argsort(u)
    out = np.empty(u.size, np.int64)
    out[order] = np.searchsorted(cumw, u[order], side="right")
    return out


def _contains(sorted_keys, q):
    """Membership of q in a sorted int64 array."""
    if sorted_keys.size == 0:
        return np.zeros(q.size, bool)
    i = np.searchsorted(sorted_keys, q)
    return sorted_keys[np.minimum(i, sorted_keys.size - 1)] == q


def _draw_excluding(rng, cumw, keys, rows, need, n):
    """For each row r of ``rows``, ``need`` more columns drawn one at a time
    from the weights (cumulative ``cumw``) restricted to the columns of
    [0, r) the row does not hold: the uniform draw u is taken on the reduced
    total and moved past the weight of every held column at or below the
    column it lands on, until the landing column no longer changes."""
    out = []
    for r, k in zip(rows.tolist(), need.tolist()):
        a, b = np.searchsorted(keys, [r * n, (r + 1) * n])
        held = sorted((keys[a:b] % n).tolist())
        for _ in range(k):
            hw = [cumw[h] - (cumw[h - 1] if h else 0.0) for h in held]
            while True:
                u = rng.random() * (cumw[r - 1] - sum(hw))
                c = -1
                for _ in range(len(held) + 2):
                    shift = sum(x for h, x in zip(held, hw) if h <= c) if c >= 0 else 0.0
                    c2 = min(int(np.searchsorted(cumw, u + shift, side="right")), r - 1)
                    if c2 == c:
                        break
                    c = c2
                if c not in held:
                    break
            held = sorted(held + [c])
            out.append(r * n + c)
    return np.array(out, np.int64)


def _leveled(widths, extra, pick, rng, name) -> Csr:
    """Rows grouped by level in natural order, level l holding widths[l] rows.
    Every row of level l >= 1 reads one random row of level l-1 (so its
    longest-path level is exactly l) plus extra(l, count) further rows drawn by
    pick(l, count) from earlier levels; duplicates are merged."""
    widths = np.asarray(widths, dtype=np.int64)
    start = np.zeros(widths.size + 1, dtype=np.int64)
    np.cumsum(widths, out=start[1:])
    rs, cs = [], []
    for lv in range(1, widths.size):
        r = np.arange(start[lv], start[lv + 1])
        rs.append(r)
        cs.append(rng.integers(start[lv - 1], start[lv], size=r.size))
        k = extra(lv, r.size)
        if k.sum():
            rs.append(np.repeat(r, k))
            cs.append(pick(lv, int(k.sum())))
    rows = np.concatenate(rs)
    cols = np.concatenate(cs)
    key = np.unique(rows * int(start[-1]) + cols)
    return _assemble(int(start[-1]), key // int(start[-1]), key % int(start[-1]), rng, name)


def lung2_like(seed: int = 0, fat_rows: int = 108_554, fat_levels: int = 26, two_row_levels: int = 453,
               extra_mean: float = 2.646) -> Csr:
    """Stand-in for SuiteSparse lung2 from its published statistics only
    (Sec. IV, Table I: n = 109,460, nnz = 492,564, 479 levels of which 453
    hold 2 rows): a fat head of ``fat_levels`` levels, each row reading one
    row of the level before and Poisson(extra_mean) rows of the three levels
    before, then ``two_row_levels`` levels of 2 rows, each row reading a row of
    the level before and one row of the head."""
    rng = np.random.default_rng(seed)
    base, rem = divmod(fat_rows, fat_levels)
    widths = [base + (1 if i < rem else 0) for i in range(fat_levels)] + [2] * two_row_levels
    start = np.concatenate([[0], np.cumsum(widths)])

    def extra(lv, cnt):
        if lv < fat_levels:
            return rng.poisson(extra_mean, size=cnt)
        return np.ones(cnt, dtype=np.int64)

    def pick(lv, cnt):
        if lv < fat_levels:
            return rng.integers(start[max(0, lv - 3)], start[lv], size=cnt)
        return rng.integers(0, start[fat_levels], size=cnt)

    return _leveled(widths, extra, pick, rng, f"lung2_like_s{seed}")


def torso2_like(seed: int = 0, n: int = 115_967, nlev: int = 513, extra_mean: float = 7.8, spread: int = 2,
                back: int = 8) -> Csr:
    """Stand-in for SuiteSparse torso2 from its published statistics only
    (Sec. IV, Table I: n = 115,967, nnz = 1,033,473, 513 levels, a triangular
    profile of rows per level). torso2 is a mesh model, so coupling is local:
    a row at relative position f of its level reads the row near f (within
    +-``spread``) of the level before, plus Poisson(extra_mean) rows near f of
    levels drawn uniformly from the ``back`` levels before."""
    rng = np.random.default_rng(seed)
    tri = np.minimum(np.arange(1, nlev + 1), np.arange(nlev, 0, -1)).astype(np.float64)
    widths = np.maximum(1, np.floor(tri * (n / tri.sum()))).astype(np.int64)
    widths[nlev // 2] += n - int(widths.sum())
    start = np.concatenate([[0], np.cumsum(widths)])

    def near(src, f):
        pos = np.floor(f * widths[src]).astype(np.int64) + rng.integers(-spread, spread + 1, size=f.size)
        return start[src] + np.clip(pos, 0, widths[src] - 1)

    rs, cs = [], []
    for lv in range(1, nlev):
        w = int(widths[lv])
        r = np.arange(start[lv], start[lv + 1])
        f = (np.arange(w) + 0.5) / w
        rs.append(r)
        cs.append(near(np.full(w, lv - 1), f))  # fixes the row's level at lv
        k = rng.poisson(extra_mean, size=w)
        if k.sum():
            src = lv - rng.integers(1, min(back, lv) + 1, size=int(k.sum()))
            rs.append(np.repeat(r, k))
            cs.append(near(src, np.repeat(f, k)))
    key = np.unique(np.concatenate(rs) * n + np.concatenate(cs))
    return _assemble(n, key // n, key % n, rng, f"torso2_like_s{seed}")


def policy_training_matrix(seed: int) -> Csr:
    """One matrix of the learned policy's training or held-out set: power-law
    recipe with n ~ U[50k, 500k], local window ~ U{256..4096} and 0-16
    near-serial segments of 250 rows, all drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50_000, 500_001))
    w_loc = int(rng.integers(256, 4097))
    nseg = int(rng.integers(0, 17))
    return powerlaw(n, seed, w_loc=w_loc, nseg=nseg, seglen=250)


def batch_window(nmat: int = 512, seed: int = 3, nmin: int = 1000, nmax: int = 50000,
                 window: int = 64) -> list[Csr]:
    """``nmat`` independent window matrices with n ~ U{nmin..nmax}; matrix i
    uses the window recipe with seed 1000*seed + i."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=nmat)
    return [window_random(int(sizes[i]), 1000 * seed + i, window) for i in range(nmat)]


def rhs(m: Csr, nrhs: int = 1) -> np.ndarray:
    """U(-1,1) right-hand sides continuing the matrix's generator; returned
    column-major as an array of shape (nrhs, n) (column c is ``b[c]``)."""
    rng = np.random.default_rng(12345)
    if m.rng_state is not None:  # hand-built fixtures carry no generator state
        rng.bit_generator.state = m.rng_state
    return rng.uniform(-1.0, 1.0, size=(nrhs, m.n))


def from_dense_lower(a: np.ndarray, name: str = "dense") -> Csr:
    """CSR of the nonzero lower triangle of a dense array (diagonal kept
    even when zero, so validation can see it)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    rp = [0]
    cols, vals = [], []
    for i in range(n):
        for j in range(i):
            if a[i, j] != 0.0:
                cols.append(j)
                vals.append(a[i, j])
        cols.append(i)
        vals.append(a[i, i])
        rp.append(len(cols))
    return Csr(n, np.array(rp, np.int32), np.array(cols, np.int32), np.array(vals, np.float64), name,
               np.random.default_rng(0).bit_generator.state)


def transpose(m: Csr) -> Csr:
    """The transpose (an upper-triangular CSR for a lower input, diagonal first
    in each row), by a counting sort of the entries on their column."""
    n = m.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(m.row_ptr))
    order = np.lexsort((rows, m.col))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(m.col, minlength=n), out=rp[1:])
    return Csr(n, rp.astype(np.int32), rows[order].astype(np.int32), m.val[order].copy(), m.name + "^T")


def diagonal(n: int, seed: int = 0) -> Csr:
    return _assemble(n, np.zeros(0, np.int64), np.zeros(0, np.int64), np.random.default_rng(seed),
                     f"diag_n{n}_s{seed}")


def bidiagonal(n: int, seed: int = 0) -> Csr:
    r = np.arange(1, n, dtype=np.int64)
    return _assemble(n, r, r - 1, np.random.default_rng(seed), f"bidiag_n{n}_s{seed}")


def config_matrix(idx: int, scale: str = "full"):
    """The synthetic workload of each configuration.

    ``scale="full"`` gives the benchmark sizes; ``scale="small"`` gives shapes
    of the same structure small enough for the serial oracle in a test.
    Returns (matrix or list of matrices, nrhs)."""
    small = scale == "small"
    if idx == 0:
        return window_random(2000, 0), 1
    if idx == 1:
        return (stencil2d_chain(48, 600, 1) if small else stencil2d_chain(1000, 20000, 1)), 1
    if idx == 2:
        if small:
            return powerlaw(60_000, 2, w_loc=512, nseg=4, seglen=60), 1
        return powerlaw(4_000_000, 2), 1
    if idx == 3:
        if small:
            return batch_window(12, 3, 500, 3000), 16
        return batch_window(512, 3), 16
    if idx == 4:
        return (stencil3d_tail(16, 300, 4) if small else stencil3d_tail(200, 5000, 4)), 32
    raise ValueError(idx)
