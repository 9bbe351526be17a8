"""The rewriting strategies the paper compares, as presets of sptrsv_rewrite,
and a Table-I-style report.

Strategies (Sec. III and the comparison of Sec. IV):
  none          no rewriting
  avgLevelCost  the paper's strategy: a level is thin when its cost is below
                avgLevelCost, and rows are moved into a target level while its
                cost stays within avgLevelCost (Sec. III)
  manual10      the comparison approach of Sec. IV: the levels cheaper than
                avgLevelCost are taken in order, ten at a time; the first of
                each ten is the target and the other nine are rewritten into
                it as whole levels (distance at most 9, no cost or fill limit)
  avgLevelCost_indeg4
                avgLevelCost with the first row constraint of Sec. III.A: a
                row is rewritten only if its rewritten form has fewer than 4
                dependencies (otherwise it stays, and the run goes on)
  naive32       this library's benchmark rule: levels with fewer than 32 rows,
                at most 32 rows per target, fill at most 4x per row

    python -m paper_2206_05843_amd.strategies --out DIR [--reps 20]

writes report.json (per matrix and strategy: levels, total and average level
cost, rows rewritten, nnz of L' and T, maximum distance, autotuned solve time,
per-level costs) and report.md (the table) for the lung2-like and torso2-like
stand-in matrices. Every rewritten solution is checked against the plain
solution of the same right-hand side (relative error <= 1e-10) and the plain
one by its residual.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2206_05843_amd import sptrsv as sp  # noqa: E402

STRATEGIES = ("none", "avgLevelCost", "avgLevelCost_indeg4", "manual10", "naive32")


def manual_mask(h: sp.Handle) -> torch.Tensor:
    """Source levels of the manual approach (Sec. IV): among the levels whose
    cost is below avgLevelCost (level 0 excluded), counted in order from 0,
    every one whose count is not a multiple of ten. The others stay targets,
    as do all levels at or above avgLevelCost."""
    st = h.level_stats(sp.ORIGINAL)
    thin = st["cost"].to(torch.float64) < st["avg"]
    thin[0] = False
    rank = torch.cumsum(thin.to(torch.int64), 0) - 1
    return (thin & (rank % 10 != 0)).to(torch.uint8)


def apply(h: sp.Handle, name: str):
    """Rewrite h with the named strategy; returns the rewrite statistics (None
    for 'none')."""
    if name == "none":
        return None
    if name == "avgLevelCost":
        return h.rewrite(sp.THIN_COST, 0.0, 0.0, 0)
    if name == "avgLevelCost_indeg4":
        return h.rewrite(sp.THIN_COST, 0.0, 0.0, 0, max_indegree=4)
    if name == "manual10":
        return h.rewrite(sp.THIN_COST, 1e300, 0.0, 9, manual_mask(h))
    if name == "naive32":
        return h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
    raise ValueError(name)


def _time(h, which, b, reps):
    h.autotune(which, 1)
    x = h.solve(b, which)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        h.solve(b, which, x)
    torch.cuda.synchronize()
    h.check()
    return (time.perf_counter() - t) / reps * 1e3, x


def report(matrices, reps: int = 20):
    out = []
    for m, b_np in matrices:
        d = torch.device("cuda")
        rp, ci, va = (torch.from_numpy(a).to(d) for a in (m.row_ptr, m.col, m.val))
        b = torch.from_numpy(b_np).to(d)
        xr = None
        for name in STRATEGIES:
            h = sp.Handle()
            h.analyze(rp, ci, va)
            st = apply(h, name)
            which = sp.ORIGINAL if st is None else sp.REWRITTEN
            cost = h.level_stats(which)
            ms, x = _time(h, which, b, reps)
            if xr is None:
                xr = x.clone()
                res = max(h.residual(b, x))
                assert res <= 1e-12 * (1.0 + float(x.abs().max())), (m.name, "residual", res)
            else:
                err = float((x - xr).abs().max() / xr.abs().max())
                assert err <= 1e-10, (m.name, name, err)
            row = {"matrix": m.name, "n": m.n, "nnz": m.nnz, "strategy": name, "levels": len(cost["cost"]),
                   "total_cost": int(cost["total"]), "avg_level_cost": float(cost["avg"]),
                   "rows_rewritten": 0 if st is None else st["rows_rewritten"],
                   "rows_held": 0 if st is None else st["rows_skipped"],
                   "nnz_Lp": m.nnz if st is None else st["nnz_Lp"], "nnz_T": m.n if st is None else st["nnz_T"],
                   "max_distance": 0 if st is None else st["max_distance"], "solve_ms": ms,
                   "level_costs": cost["cost"].cpu().numpy().tolist()}
            out.append(row)
            print(f"[strategies] {m.name} {name}: levels {row['levels']} avg cost {row['avg_level_cost']:.1f} "
                  f"total {row['total_cost']} rewritten {row['rows_rewritten']} solve {ms:.3f} ms", flush=True)
            h.close()
    return out


def profile(costs, bins: int = 16):
    """Per-level costs in the manner of Figs. 5 and 6: the levels cut into
    `bins` consecutive groups of (nearly) equal size, each group's mean and
    largest level cost, and the largest level cost overall."""
    c = np.asarray(costs, dtype=np.float64)
    edges = np.linspace(0, c.size, min(bins, c.size) + 1).astype(int)
    return {"mean": [float(c[a:b].mean()) for a, b in zip(edges[:-1], edges[1:])],
            "max": [float(c[a:b].max()) for a, b in zip(edges[:-1], edges[1:])],
            "peak": float(c.max()), "levels_over_avg": int((c > c.mean()).sum())}


def markdown(rows) -> str:
    lines = ["| matrix | strategy | levels | avg level cost | total level cost | rows rewritten | rows held | nnz(L') | "
             "nnz(T) | max distance | solve ms |", "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {r['matrix']} | {r['strategy']} | {r['levels']} | {r['avg_level_cost']:.1f} | "
                     f"{r['total_cost']} | {r['rows_rewritten']} | {r.get('rows_held', 0)} | {r['nnz_Lp']} | {r['nnz_T']} | "
                     f"{r['max_distance']} | {r['solve_ms']:.3f} |")
    lines += ["", "Per-level cost profile (as in Figs. 5 and 6): the levels in 16 consecutive groups, each group's mean "
              "level cost, then the largest level cost and the number of levels above the average.", "",
              "| matrix | strategy | mean cost per group of levels | largest | levels > avg |", "|---|---|---|---|---|"]
    for r in rows:
        pr = profile(r["level_costs"])
        lines.append(f"| {r['matrix']} | {r['strategy']} | {' '.join(f'{v:.0f}' for v in pr['mean'])} | "
                     f"{pr['peak']:.0f} | {pr['levels_over_avg']} |")
    return "\n".join(lines) + "\n"


def main():
    import gen
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    mats = []
    for f in (gen.lung2_like, gen.torso2_like):
        m = f(0)
        mats.append((m, gen.rhs(m, 1)[0]))
    rows = report(mats, args.reps)
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(rows, f)
    with open(os.path.join(args.out, "report.md"), "w") as f:
        f.write(markdown(rows))


if __name__ == "__main__":
    main()
