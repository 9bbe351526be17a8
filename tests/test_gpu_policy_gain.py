"""Held-out gain of the shipped learned policy on power-law matrices.

Seeds 2000-2019 of the policy's matrix family (n ~ U[50k, 500k]) are used
neither in training (1000-1199) nor in choosing the action and the tier
thresholds (1900-1909). On each, plain, naive (thin levels < 32 rows, budget
32, fill cap 4x) and learned are autotuned and timed (median of 21 solves
between HIP events); the plain solution is checked against the oracle and
each rewritten one against the plain one (relative error <= 1e-10). The
geometric mean of naive time / learned time over the seeds must exceed 1.02:
the network's per-level choice of what to rewrite, and how far, has to beat
the thin-level rule (Sec. III.A)."""
import json
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import dev, to_dev

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2206_05843_amd")

SEEDS = list(range(2000, 2020))
TOL = 1e-10
_RES = {}


def _time(h, which, b, reps=21):
    h.autotune(which, 1)
    x = torch.empty_like(b)
    for _ in range(3):
        h.solve(b, which, x)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        h.solve(b, which, x)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    h.check()
    return float(np.median(ts)), x


@pytest.mark.parametrize("seed", SEEDS)
def test_heldout_seed(seed):
    from paper_2206_05843_amd import policy
    pol = policy.load_default()
    assert pol is not None, "no policy checkpoint"
    m = gen.policy_training_matrix(seed)
    b_np = gen.rhs(m, 1)
    b = to_dev(b_np[0])
    res = {"n": m.n}
    xr = None
    for name in ("plain", "naive", "learned"):
        h = sp.Handle()
        h.analyze(*dev(m))
        which = sp.ORIGINAL
        if name == "naive":
            st = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
            which = sp.REWRITTEN
        elif name == "learned":
            st = policy.rewrite_learned(h, pol)
            which = sp.REWRITTEN
        ms, x = _time(h, which, b)
        if xr is None:
            xr = x.clone()
            assert oracle.relerr(x.cpu().numpy()[None], oracle.solve(m, b_np)) <= TOL
        else:
            assert float((x - xr).abs().max() / xr.abs().max()) <= TOL, name
        res[name] = ms
        if which == sp.REWRITTEN:
            res[name + "_nlev"] = st["nlev_after"]
        h.close()
    _RES[seed] = res
    print(f"seed {seed}: {json.dumps(res)}")


def test_heldout_geomean(tmp_path_factory):
    if len(_RES) != len(SEEDS):
        pytest.skip("needs every held-out seed in the same run")
    g = {k: math.exp(np.mean([math.log(r[k] / r["learned"]) for r in _RES.values()])) for k in ("naive", "plain")}
    out = tmp_path_factory.mktemp("gain") / "policy_heldout.json"
    out.write_text(json.dumps({"geomean_naive_over_learned": g["naive"], "geomean_plain_over_learned": g["plain"],
                               "per_seed": _RES}, indent=1))
    print(f"held-out geomean: learned vs naive x{g['naive']:.4f}, vs plain x{g['plain']:.4f} ({out})")
    assert g["naive"] > 1.02
    assert g["plain"] > 1.0
