"""GPU parity of the paper's rewriting strategies (Sec. III avgLevelCost, the
Sec. IV manual distance-10 approach, the naive rule) on the lung2-like and
torso2-like stand-ins: rewritten patterns, values and targets bit for bit,
Table I metrics equal to the oracle's, and x within 1e-10."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")
from paper_2206_05843_amd import strategies  # noqa: E402


def _manual_sources(m, lv):
    # levels cheaper than avgLevelCost (level 0 excluded), ten at a time: the
    # first of each ten is kept as the target, the other nine are sources
    c = oracle.level_costs(m, lv)
    thin = c.cost.astype(np.float64) < c.avg
    thin[0] = False
    rank = np.cumsum(thin) - 1
    return (thin & (rank % 10 != 0)).astype(np.uint8)


def _oracle_rewrite(m, name, lv):
    if name == "avgLevelCost":
        return oracle.rewrite(m, oracle.THIN_COST, 0.0, 0.0, 0, lv=lv)
    if name == "manual10":
        return oracle.rewrite(m, oracle.THIN_COST, 1e300, 0.0, 9, mask=_manual_sources(m, lv), lv=lv)
    if name == "avgLevelCost_indeg4":
        return oracle.rewrite(m, oracle.THIN_COST, 0.0, 0.0, 0, lv=lv, max_indegree=4)
    if name == "naive32":
        return oracle.rewrite(m, oracle.THIN_ROWS, 32.0, 4.0, 0, lv=lv)
    raise ValueError(name)


@pytest.mark.parametrize("mk", [gen.lung2_like, gen.torso2_like])
@pytest.mark.parametrize("name", ["avgLevelCost", "avgLevelCost_indeg4", "manual10", "naive32"])
def test_strategy_parity(mk, name):
    m = mk(0)
    lv = oracle.levels(m)
    h = sp.Handle()
    h.analyze(*dev(m))
    if name == "manual10":
        assert np.array_equal(strategies.manual_mask(h).cpu().numpy(), _manual_sources(m, lv))
    st = strategies.apply(h, name)
    rw = _oracle_rewrite(m, name, lv)
    g = {k: v.cpu().numpy() for k, v in h.rewritten().items()}
    assert np.array_equal(g["lp_ptr"], rw.lp_ptr) and np.array_equal(g["lp_col"], rw.lp_col)
    assert np.array_equal(g["lp_val"], rw.lp_val)
    assert np.array_equal(g["t_ptr"], rw.t_ptr) and np.array_equal(g["t_col"], rw.t_col)
    assert np.array_equal(g["t_val"], rw.t_val)
    assert np.array_equal(h.targets().cpu().numpy(), rw.target)
    ref = oracle.rewrite_stats(m, rw, lv)
    for k in ("nlev_before", "nlev_after", "rows_rewritten", "max_distance", "nnz_Lp", "nnz_T"):
        assert st[k] == ref[k], k
    assert st["rows_skipped"] == rw.rows_skipped
    for k in ("total_cost_before", "total_cost_after", "avg_level_cost_before", "avg_level_cost_after"):
        assert st[k] == ref[k], k
    b = gen.rhs(m, 1)
    x = h.solve(to_dev(b[0]), sp.REWRITTEN)
    h.check()
    assert oracle.relerr(x.cpu().numpy(), oracle.solve(m, b)) <= 1e-10
