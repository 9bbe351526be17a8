"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark times (each variant autotuned first): levels bit for bit, every
output of x within relative 1e-10 of the oracle, rewritten patterns and values
bit for bit, and the whole batch of matrices."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

TOL = 1e-10
FULL = [1, 2, 4]


@pytest.fixture(scope="module")
def full():
    out = {}
    for c in FULL:
        m, nrhs = gen.config_matrix(c)
        b = gen.rhs(m, nrhs)
        out[c] = (m, nrhs, b, oracle.solve(m, b))
    return out


@pytest.mark.parametrize("cfg", FULL)
def test_full_levels(full, cfg):
    m = full[cfg][0]
    h = sp.Handle()
    nlev = h.analyze(*dev(m))
    lv = oracle.levels(m)
    assert nlev == lv.nlev
    lp, lr, rl = (t.cpu().numpy() for t in h.levels())
    assert np.array_equal(lp, lv.level_ptr) and np.array_equal(lr, lv.level_rows)
    assert np.array_equal(rl, lv.row_level)


@pytest.mark.parametrize("cfg", FULL)
@pytest.mark.parametrize("variant", ["plain", "naive", "learned"])
def test_full_solve_autotuned(full, cfg, variant):
    m, nrhs, b, xr = full[cfg]
    h = sp.Handle()
    h.analyze(*dev(m))
    which = sp.ORIGINAL
    if variant == "naive":
        h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
        which = sp.REWRITTEN
    elif variant == "learned":
        from paper_2206_05843_amd import policy
        policy.rewrite_learned(h, policy.load_default())
        which = sp.REWRITTEN
    h.autotune(which, nrhs)
    bd = to_dev(b)
    x = h.solve(bd if nrhs > 1 else bd.view(-1), which)
    h.check()
    assert oracle.relerr(x.view(nrhs, -1).cpu().numpy(), xr) <= TOL
    # a second solve into the same buffers gives the same bits
    x2 = h.solve(bd if nrhs > 1 else bd.view(-1), which)
    assert torch.equal(x, x2)


@pytest.mark.parametrize("variant", ["plain", "naive"])
def test_full_solve_rows_graph(full, variant):
    """The 3D stencil workload as the benchmark times it: right-hand sides by
    rows, tuned by rows, solved in hipGraph replays; every output against the
    oracle, every replay bit for bit the eager solve."""
    m, nrhs, b, xr = full[4]
    h = sp.Handle()
    h.analyze(*dev(m))
    which = sp.ORIGINAL
    if variant == "naive":
        h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
        which = sp.REWRITTEN
    h.autotune(which, nrhs, rows=True)
    print(f"full rows: {variant} schedule={h.get_schedule(which, nrhs)}", flush=True)
    br = to_dev(b).t().contiguous()
    x = h.solve_rows(br, which)
    h.check()
    assert oracle.relerr(x.t().cpu().numpy(), xr) <= TOL
    xg = torch.zeros_like(x)
    st = torch.cuda.Stream()  # graph capture needs a non-default stream
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        gid = h.graph_create_rows(br, xg, which)
        for _ in range(3):
            xg.zero_()
            h.graph_launch(gid)
            st.synchronize()
            assert torch.equal(xg, x)
        h.check()


def _oracle_policy_actions(m, lv, pol):
    """The shipped policy's per-level actions computed on the CPU side: the
    oracle's FP64 features through the FP64 network with the checkpoint's
    weights (rounded to the float32 the checkpoint holds), then the highest
    tier whose threshold the probability reaches. Also returns the oracle's
    probabilities, to find decisions that sit on a threshold."""
    from oracle import mlp
    th = pol.params.cpu().numpy().astype(np.float64)
    norm = pol.norm.cpu().numpy().astype(np.float64)
    fo = oracle.level_features(m, lv)
    po, _ = mlp.forward(th, (fo - norm[:mlp.F_IN]) * norm[mlp.F_IN:])
    tier = np.full(lv.nlev, -1)
    for j, (t, _, _) in enumerate(pol.tiers):
        tier[po >= t] = j
    tier[0] = -1
    mask = (tier >= 0).astype(np.uint8)
    budget = np.array([pol.tiers[k][1] if k >= 0 else 0 for k in tier], np.int32)
    cap = np.array([pol.tiers[k][2] if k >= 0 else 0.0 for k in tier], np.float32)
    return mask, budget, cap, po


def _same_rewrite(h, rw):
    g = {k: v.cpu().numpy() for k, v in h.rewritten().items()}
    assert np.array_equal(g["lp_ptr"], rw.lp.row_ptr) and np.array_equal(g["lp_col"], rw.lp.col)
    assert np.array_equal(g["t_ptr"], rw.t_ptr) and np.array_equal(g["t_col"], rw.t_col)
    assert np.array_equal(g["lp_val"], rw.lp.val) and np.array_equal(g["t_val"], rw.t_val)
    assert np.array_equal(h.targets().cpu().numpy(), rw.target)


@pytest.mark.parametrize("cfg,variant", [(1, "naive"), (2, "naive"), (1, "learned"), (2, "learned")])
def test_full_rewrite_patterns(full, cfg, variant):
    """Rewritten L', T and targets at full size, bit for bit. For the learned
    variant the per-level actions (mask, target budget, fill cap) are the CPU
    side's (the oracle's features and network); the device's own actions must
    agree with them on every level whose oracle probability is not within 1e-4
    of a threshold."""
    m = full[cfg][0]
    lv = oracle.levels(m)
    h = sp.Handle()
    h.analyze(*dev(m))
    mask = budget = cap = None
    if variant == "learned":
        from paper_2206_05843_amd import policy
        pol = policy.load_default()
        assert pol is not None
        mask, budget, cap, po = _oracle_policy_actions(m, lv, pol)
        gm, gb, gc = (a.cpu().numpy() for a in pol.actions(h))
        sure = np.all([np.abs(po - t) > 1e-4 for t, _, _ in pol.tiers], axis=0)
        assert np.array_equal(gm[sure], mask[sure])
        assert np.array_equal(gb[sure], budget[sure]) and np.array_equal(gc[sure], cap[sure])
    st = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0, to_dev(mask) if mask is not None else None,
                   level_budget=to_dev(budget) if budget is not None else None,
                   level_fill_cap=to_dev(cap) if cap is not None else None)
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, mask, lv, level_budget=budget, level_cap=cap)
    assert st["rows_rewritten"] == rw.rows_rewritten
    assert st["nlev_after"] == oracle.levels(rw.lp).nlev
    _same_rewrite(h, rw)


def test_full_rewrite_patterns_3d():
    m = gen.config_matrix(4)[0]
    h = sp.Handle()
    h.analyze(*dev(m))
    st = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
    rw = oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0)
    assert st["nlev_after"] == oracle.levels(rw.lp).nlev
    g = {k: v.cpu().numpy() for k, v in h.rewritten().items()}
    assert np.array_equal(g["lp_ptr"], rw.lp.row_ptr) and np.array_equal(g["lp_col"], rw.lp.col)
    assert np.array_equal(g["t_ptr"], rw.t_ptr) and np.array_equal(g["t_col"], rw.t_col)
    assert np.array_equal(g["lp_val"], rw.lp.val) and np.array_equal(g["t_val"], rw.t_val)
    assert np.array_equal(h.targets().cpu().numpy(), rw.target)


def test_full_batch():
    mats, nrhs = gen.config_matrix(3)
    h = sp.Handle()
    h.batch_analyze([m.n for m in mats], to_dev(np.concatenate([m.row_ptr for m in mats]).astype(np.int32)),
                    to_dev(np.concatenate([m.col for m in mats])), to_dev(np.concatenate([m.val for m in mats])))
    bs = [gen.rhs(m, nrhs) for m in mats]
    b = to_dev(np.concatenate([x.reshape(-1) for x in bs]))
    x = torch.zeros_like(b)
    h.batch_solve(b, x, nrhs)
    h.check()
    xs = x.cpu().numpy()
    off = 0
    for i, (m, bm) in enumerate(zip(mats, bs)):
        assert oracle.relerr(xs[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n), oracle.solve(m, bm)) <= TOL
        if i % 64 == 0:  # levels of a sample of the matrices
            lp, lr = h.batch_levels(i)
            lv = oracle.levels(m)
            assert np.array_equal(lp.cpu().numpy(), lv.level_ptr) and np.array_equal(lr.cpu().numpy(), lv.level_rows)
        off += m.n
