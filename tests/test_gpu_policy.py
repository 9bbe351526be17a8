"""GPU parity of the learned policy's kernels: level features against the
oracle's, and the network's forward, backward (gradients) and Adam against
the FP64 network oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import mlp
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")


@pytest.mark.parametrize("mk", [lambda: gen.config_matrix(0)[0], lambda: gen.config_matrix(1, "small")[0],
                                lambda: gen.config_matrix(2, "small")[0], lambda: gen.window_random(3000, 5, 30, 9)])
def test_features_match_oracle(mk):
    m = mk()
    h = sp.Handle()
    h.analyze(*dev(m))
    f = h.level_features().cpu().numpy().astype(np.float64)
    fo = oracle.level_features(m)
    np.testing.assert_allclose(f, fo, rtol=2e-6, atol=1e-6)


def _batch(seed, B=300):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(B, mlp.F_IN))
    y = (rng.random(B) < 0.3).astype(np.float64)
    th = mlp.init(seed) + rng.normal(scale=0.05, size=mlp.NPARAM)
    return th.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64), y


def test_forward_matches_oracle():
    th, f, _ = _batch(1)
    p = sp.mlp_forward(to_dev(th, torch.float32), to_dev(f, torch.float32)).cpu().numpy()
    po, _ = mlp.forward(th, f)
    np.testing.assert_allclose(p, po, rtol=1e-5, atol=1e-6)


def test_forward_normalisation():
    th, f, _ = _batch(2)
    mean = np.linspace(-1, 1, mlp.F_IN)
    inv = np.linspace(0.5, 2, mlp.F_IN)
    norm = np.concatenate([mean, inv]).astype(np.float32)
    p = sp.mlp_forward(to_dev(th, torch.float32), to_dev(f, torch.float32), to_dev(norm)).cpu().numpy()
    fz = (f - norm[:mlp.F_IN].astype(np.float64)) * norm[mlp.F_IN:].astype(np.float64)
    po, _ = mlp.forward(th, fz)
    np.testing.assert_allclose(p, po, rtol=2e-5, atol=1e-6)


@pytest.mark.parametrize("B", [1, 7, 300, 1100])
def test_backward_matches_oracle(B):
    th, f, y = _batch(3, B)
    g, loss = sp.mlp_backward(to_dev(th, torch.float32), to_dev(f, torch.float32), to_dev(y, torch.float32))
    go, lo = mlp.backward(th, f, y)
    g = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    np.testing.assert_allclose(g, go, rtol=1e-3, atol=1e-6 * np.abs(go).max())
    assert abs(float(loss) - lo) <= 1e-5 * abs(lo)


def test_backward_weights_and_determinism():
    th, f, y = _batch(4)
    P, F, Y = to_dev(th, torch.float32), to_dev(f, torch.float32), to_dev(y, torch.float32)
    g1, l1 = sp.mlp_backward(P, F, Y)
    g2, l2 = sp.mlp_backward(P, F, Y, weight=torch.ones_like(Y))
    g3, _ = sp.mlp_backward(P, F, Y)
    assert torch.equal(g1, g3)  # fixed reduction order
    assert torch.allclose(g1, g2) and torch.allclose(l1, l2)
    g4, l4 = sp.mlp_backward(P, F, Y, weight=2 * torch.ones_like(Y))
    assert torch.allclose(g4, 2 * g1, rtol=1e-6, atol=1e-9) and torch.allclose(l4, 2 * l1)


def test_adam_matches_oracle():
    th, f, y = _batch(5)
    P = to_dev(th, torch.float32)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    tho, mo, vo = th.copy(), np.zeros_like(th), np.zeros_like(th)
    F, Y = to_dev(f, torch.float32), to_dev(y, torch.float32)
    for step in range(1, 6):
        g, _ = sp.mlp_backward(P, F, Y)
        go = g.cpu().numpy().astype(np.float64)  # same gradient for both updates
        sp.mlp_adam(P, g, m, v, step, 1e-3)
        tho, mo, vo = mlp.adam(tho, go, mo, vo, step, 1e-3)
    np.testing.assert_allclose(P.cpu().numpy(), tho, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss_on_separable_data():
    rng = np.random.default_rng(9)
    f = rng.normal(size=(512, mlp.F_IN)).astype(np.float32)
    y = (f[:, 0] + 0.5 * f[:, 3] > 0).astype(np.float32)
    P = to_dev(mlp.init(0), torch.float32)
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    F, Y = to_dev(f), to_dev(y)
    losses = []
    for step in range(1, 201):
        g, loss = sp.mlp_backward(P, F, Y)
        sp.mlp_adam(P, g, m, v, step, 3e-3)
        losses.append(float(loss))
    assert losses[-1] < 0.2 * losses[0]
    acc = ((sp.mlp_forward(P, F) >= 0.5).float() == Y).float().mean()
    assert float(acc) > 0.95


def test_mask():
    p = torch.tensor([0.9, 0.2, 0.5, 0.7, 0.49], device="cuda")
    assert sp.mlp_mask(p, 0.5).cpu().tolist() == [0, 0, 1, 1, 0]


def test_level_times():
    m = gen.config_matrix(1, "small")[0]
    h = sp.Handle()
    nlev = h.analyze(*dev(m))
    b = to_dev(gen.rhs(m, 1)[0])
    t = h.level_times(b).cpu().numpy()
    assert t.shape == (nlev,) and np.all(t >= 0) and t.sum() > 0
    x = h.solve(b)  # ordinary solves still right after a timed run
    assert oracle.relerr(x.cpu().numpy()[None], oracle.solve(m, b.cpu().numpy()[None])) <= 1e-10


@pytest.mark.parametrize("knobs", [dict(max_indegree=4), dict(max_spread=64), dict(critical_only=True)])
def test_learned_rewrite_with_row_constraints(knobs):
    """rewrite_learned with the Sec. III.A row constraints as knobs: the level
    mask of a (random-weight) policy equals the FP64 oracle network's on the
    oracle's features, with the threshold in the widest gap of the oracle's
    probabilities so that no decision sits on the rounding edge, and the
    rewritten matrices equal the oracle's rewrite with that mask and the same
    constraints."""
    from paper_2206_05843_amd import policy
    m = gen.window_random(3000, 5, 30, 9)
    lv = oracle.levels(m)
    th = mlp.init(4)
    fo = oracle.level_features(m, lv)
    mean, sd = fo.mean(axis=0), fo.std(axis=0) + 1e-3
    norm = np.concatenate([mean, 1.0 / sd]).astype(np.float32)
    po, _ = mlp.forward(th.astype(np.float32).astype(np.float64),
                        (fo - norm[:mlp.F_IN].astype(np.float64)) * norm[mlp.F_IN:].astype(np.float64))
    q = np.sort(po[1:])
    k = int(np.argmax(np.diff(q)))
    thr = float((q[k] + q[k + 1]) / 2)
    assert q[k + 1] - q[k] > 1e-3
    mask = ((po >= thr) & (np.arange(lv.nlev) > 0)).astype(np.uint8)
    pol = policy.Policy(th, norm, thr)
    h = sp.Handle()
    h.analyze(*dev(m))
    assert np.array_equal(pol.mask_for(h).cpu().numpy(), mask)
    st = policy.rewrite_learned(h, pol, **knobs)
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, mask, lv, **knobs)
    g = {k2: v.cpu().numpy() for k2, v in h.rewritten().items()}
    assert np.array_equal(g["lp_ptr"], rw.lp.row_ptr) and np.array_equal(g["lp_col"], rw.lp.col)
    assert np.array_equal(g["t_ptr"], rw.t.row_ptr) and np.array_equal(g["t_col"], rw.t.col)
    assert st["rows_skipped"] == rw.rows_skipped


def test_mlp_actions_tiers():
    """Tiered actions from probabilities: the highest tier whose threshold
    the probability reaches, level 0 never a source (direct definition)."""
    rng = np.random.default_rng(11)
    p = rng.random(1000).astype(np.float32)
    p[[5, 6, 7]] = [0.2, 0.6, 0.59999]
    tiers = [(0.2, 0, 0.0), (0.6, 128, 8.0)]
    mask, bud, cap = (a.cpu().numpy() for a in sp.mlp_actions(to_dev(p), tiers))
    k = np.where(p >= 0.6, 1, np.where(p >= 0.2, 0, -1))
    k[0] = -1
    assert np.array_equal(mask, (k >= 0).astype(np.uint8))
    assert np.array_equal(bud, np.where(k == 1, 128, 0).astype(np.int32))
    assert np.array_equal(cap, np.where(k == 1, 8.0, 0.0).astype(np.float32))
    assert mask[5] == 1 and bud[5] == 0 and bud[6] == 128 and bud[7] == 0
    # one tier reproduces sptrsv_mlp_mask
    m1, _, _ = sp.mlp_actions(to_dev(p), [(0.5, 0, 0.0)])
    assert torch.equal(m1, sp.mlp_mask(to_dev(p), 0.5))
    with pytest.raises(sp.SptrsvError):
        sp.mlp_actions(to_dev(p), [(0.6, 0, 0.0), (0.2, 64, 4.0)])  # thresholds out of order
    with pytest.raises(sp.SptrsvError):
        sp.mlp_actions(to_dev(p), [(0.1, -1, 0.0)])
    with pytest.raises(sp.SptrsvError):
        sp.mlp_actions(to_dev(p), [(0.1, 0, 0.0)] * 5)


def test_policy_tiers_rewrite_matches_oracle():
    """A two-tier policy (random weights) through rewrite_learned: mask,
    per-level budget and cap from the device equal the FP64 network's on the
    oracle's features (thresholds in wide gaps of the probabilities), and the
    rewrite equals the oracle's with those per-level actions."""
    from paper_2206_05843_amd import policy
    m = gen.config_matrix(2, "small")[0]
    lv = oracle.levels(m)
    th = mlp.init(6)
    fo = oracle.level_features(m, lv)
    mean, sd = fo.mean(axis=0), fo.std(axis=0) + 1e-3
    norm = np.concatenate([mean, 1.0 / sd]).astype(np.float32)
    po, _ = mlp.forward(th.astype(np.float32).astype(np.float64),
                        (fo - norm[:mlp.F_IN].astype(np.float64)) * norm[mlp.F_IN:].astype(np.float64))
    q = np.sort(po[1:])
    gaps = np.diff(q)
    # two thresholds in the two widest gaps between the 20% and 80% quantiles
    lo_i, hi_i = int(0.2 * len(q)), int(0.8 * len(q))
    cand = np.argsort(gaps[lo_i:hi_i])[::-1][:2] + lo_i
    t1, t2 = sorted(float((q[k] + q[k + 1]) / 2) for k in cand)
    assert min(gaps[cand]) > 1e-5
    tiers = [(t1, 0, 0.0), (t2, 96, 6.0)]
    tier = np.where(po >= t2, 1, np.where(po >= t1, 0, -1))
    tier[0] = -1
    mask = (tier >= 0).astype(np.uint8)
    budget = np.where(tier == 1, 96, 0).astype(np.int32)
    cap = np.where(tier == 1, 6.0, 0.0).astype(np.float32)
    pol = policy.Policy(th, norm, tiers)
    h = sp.Handle()
    h.analyze(*dev(m))
    gm, gb, gc = (a.cpu().numpy() for a in pol.actions(h))
    assert np.array_equal(gm, mask) and np.array_equal(gb, budget) and np.array_equal(gc, cap)
    st = policy.rewrite_learned(h, pol)
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, mask, lv, level_budget=budget, level_cap=cap)
    assert st["rows_rewritten"] == rw.rows_rewritten > 0
    g = {k2: v.cpu().numpy() for k2, v in h.rewritten().items()}
    assert np.array_equal(g["lp_ptr"], rw.lp.row_ptr) and np.array_equal(g["lp_col"], rw.lp.col)
    assert np.array_equal(g["t_ptr"], rw.t.row_ptr) and np.array_equal(g["t_col"], rw.t.col)
    assert np.array_equal(g["lp_val"], rw.lp.val) and np.array_equal(g["t_val"], rw.t.val)


def test_policy_checkpoint_roundtrip(tmp_path):
    from paper_2206_05843_amd import policy
    tiers = [(0.1, 0, 0.0), (0.4, 128, 8.0)]
    pol = policy.Policy(mlp.init(2), np.concatenate([np.zeros(mlp.F_IN), np.ones(mlp.F_IN)]), tiers, {"k": 1})
    pol.save(str(tmp_path / "p.npz"))
    q = policy.Policy.load(str(tmp_path / "p.npz"))
    assert q.tiers == pol.tiers and q.meta == {"k": 1} and torch.equal(q.params, pol.params)
    with pytest.raises(ValueError):
        policy.Policy(mlp.init(2), np.zeros(2 * mlp.F_IN), [(0.5, 0, 0.0), (0.1, 64, 4.0)])


@pytest.mark.parametrize("nrhs", [1, 3])
def test_level_finish_times(nrhs):
    """Finish times of a stamped synchronisation-free solve: on a chain
    (every level one row that reads the row before) they increase strictly
    level by level; on a general matrix a level's latest value is written
    after the earliest value of the level before it (each level >= 1 has a
    row reading a row of the level before), and every time is >= 0. Ordinary
    solves stay right afterwards."""
    ch = gen.bidiagonal(3000, 1)
    for m in (ch, gen.window_random(20000, 4, 200, 3)):
        h = sp.Handle()
        nlev = h.analyze(*dev(m))
        b = to_dev(gen.rhs(m, nrhs))
        t = h.level_finish_times(b if nrhs > 1 else b.view(-1)).cpu().numpy()
        assert t.shape == (nlev,) and np.all(np.isfinite(t)) and np.all(t >= 0)
        assert t.max() > 0
        if m is ch:
            assert np.all(np.diff(t) > 0)
        x = h.solve(b if nrhs > 1 else b.view(-1))
        h.check()
        assert oracle.relerr(x.view(nrhs, -1).cpu().numpy(), oracle.solve(m, b.view(nrhs, -1).cpu().numpy())) <= 1e-10


@pytest.mark.parametrize("use_csr", [False, True])
@pytest.mark.parametrize("mk", [lambda: gen.config_matrix(1, "small")[0], lambda: gen.policy_training_matrix(2000)])
def test_rewrite_learned_checked(mk, use_csr):
    """The measured fallback keeps either the shipped policy's rewrite or the
    naive rule's, whichever autotuned faster; the kept L' equals the oracle's
    rewrite for that choice bit for bit and the solve is right."""
    from paper_2206_05843_amd import policy
    pol = policy.load_default()
    assert pol is not None
    m = mk()
    lv = oracle.levels(m)
    h = sp.Handle()
    h.analyze(*dev(m))
    st, chosen = policy.rewrite_learned_checked(h, pol, 1, csr=dev(m) if use_csr else None)
    assert chosen in ("learned", "naive")
    if chosen == "naive":
        rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, None, lv)
    else:
        h2 = sp.Handle()
        h2.analyze(*dev(m))
        mask, bud, cap = (a.cpu().numpy() for a in pol.actions(h2))
        rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, mask, lv, level_budget=bud, level_cap=cap)
    g = {k2: v.cpu().numpy() for k2, v in h.rewritten().items()}
    assert st["rows_rewritten"] == rw.rows_rewritten
    assert np.array_equal(g["lp_ptr"], rw.lp.row_ptr) and np.array_equal(g["lp_col"], rw.lp.col)
    assert np.array_equal(g["t_ptr"], rw.t.row_ptr) and np.array_equal(g["t_col"], rw.t.col)
    b = to_dev(gen.rhs(m, 1)[0])
    x = h.solve(b, sp.REWRITTEN)
    h.check()
    assert oracle.relerr(x.cpu().numpy()[None], oracle.solve(m, b.cpu().numpy()[None])) <= 1e-10
