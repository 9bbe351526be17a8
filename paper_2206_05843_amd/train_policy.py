"""Train and evaluate the learned rewrite policy on the GPU.

    python -m paper_2206_05843_amd.train_policy --out DIR [--matrices 200] [--heldout 20]

Action. A level the network trusts becomes a source of the rewrite with a
larger target budget and fill cap than the naive strategy's (32 rows, 4x):
the pair (B, C) is chosen first, on validation matrices (seeds 1900..), as the
one whose thin-level rewrite (levels with < B rows, budget B, cap C) solves
fastest in geometric mean, each variant autotuned.

Data. For each seeded power-law training matrix (n ~ U[50k, 500k]) the
library times one synchronisation-free solve of L and one of L' after the
(B, C) rewrite -- the executor the autotuner picks on these matrices -- with
every item stamping the device clock when its value is written
(sptrsv_level_finish_times). A level's time is the growth of the running
maximum of its levels' finish times across it (its share of the critical
path). A level that the rewrite empties is labelled 1 when the time its rows
cost in their new levels of L' (their share, by row entries, of those levels'
times) is below the time the level took in L, else 0; levels that are not
emptied are labelled 0. The features are the 20 per-level features of the
original levels (sptrsv_level_features), the row constraints of Sec. III.A
among them.

Training. Mean class-balanced binary cross-entropy, Adam, minibatches; forward,
backward and the Adam step are the library's kernels. Features are
standardised with the training set's mean and standard deviation, which are
stored in the checkpoint with the weights.

Calibration. Two tiers map the network's probability to an action: p >= t_hi
takes (B, C), t_lo <= p < t_hi the naive budget and cap, p < t_lo leaves the
level alone. (t_lo, t_hi) is chosen on the validation matrices: the pair with
the best geometric-mean solve-time ratio against the naive rewrite (ties: the
pair that rewrites less).

Evaluation. On held-out seeds (2000..), plain, naive, the constant rule "(B, C)
on every thin level" and learned are autotuned and timed; the rewritten
solutions are checked against the plain solution (relative error <= 1e-10) and
the plain one by its residual. --evaluate CKPT runs only this, for a saved
checkpoint.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import gen  # noqa: E402
from paper_2206_05843_amd import sptrsv as sp  # noqa: E402
from paper_2206_05843_amd.policy import Policy, init_params  # noqa: E402

NAIVE = (32.0, 4.0)
ACTIONS = [(128, 8.0), (256, 16.0), (512, 16.0), (512, 32.0), (1024, 32.0), (1024, 64.0)]


def log(*a):
    print(*a, flush=True)


def to_dev(m):
    d = torch.device("cuda")
    return (torch.from_numpy(m.row_ptr).to(d), torch.from_numpy(m.col).to(d), torch.from_numpy(m.val).to(d))


def level_shares(finish):
    """A level's share of a synchronisation-free solve: the growth of the
    running maximum of the levels' finish times across it."""
    f = np.maximum.accumulate(np.asarray(finish, np.float64))
    return np.diff(np.concatenate([[0.0], f]))


def level_data(m, action, reps: int = 3):
    """Features, labels and time deltas of the original levels of m, under the
    rewrite with target budget and fill cap `action` on every thin level."""
    h = sp.Handle()
    h.analyze(*to_dev(m))
    feat = h.level_features().cpu().numpy()
    b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
    t_plain = np.mean([level_shares(h.level_finish_times(b, sp.ORIGINAL).cpu().numpy()) for _ in range(reps)],
                      axis=0)
    h.rewrite(sp.THIN_ROWS, float(action[0]), float(action[1]), 0)
    t_rew = np.mean([level_shares(h.level_finish_times(b, sp.REWRITTEN).cpu().numpy()) for _ in range(reps)],
                    axis=0)
    tgt = h.targets().cpu().numpy()
    rw = h.rewritten()
    work = (np.diff(rw["lp_ptr"].cpu().numpy()) - 1) + (np.diff(rw["t_ptr"].cpu().numpy()) - 1) + 1
    lev = h.levels(sp.ORIGINAL)[2].cpu().numpy()
    lev2 = h.levels(sp.REWRITTEN)[2].cpu().numpy()
    nlev = h.nlev
    wl2 = np.bincount(lev2, weights=work, minlength=t_rew.size)
    share = t_rew[lev2] * work / np.maximum(wl2[lev2], 1)
    moved = tgt >= 0
    R = np.bincount(lev, minlength=nlev)
    M = np.bincount(lev[moved], minlength=nlev)
    cost_new = np.bincount(lev, weights=share * moved, minlength=nlev)
    delta = cost_new - t_plain
    emptied = (M == R) & (np.arange(nlev) > 0)
    label = (emptied & (delta < 0)).astype(np.float32)
    valid = np.arange(nlev) > 0
    h.close()
    return feat[valid], label[valid], delta[valid], emptied[valid]


def train(feat, label, seed=0, epochs=40, batch=8192, lr=3e-3, log_every=10):
    mean = feat.mean(axis=0)
    std = feat.std(axis=0)
    std[std < 1e-6] = 1.0
    norm = np.concatenate([mean, 1.0 / std]).astype(np.float32)
    P = torch.from_numpy(init_params(seed)).to("cuda")
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    F = torch.from_numpy(feat.astype(np.float32)).to("cuda")
    Y = torch.from_numpy(label.astype(np.float32)).to("cuda")
    pos = float(label.mean())
    wpos = 0.5 / max(pos, 1e-6)
    wneg = 0.5 / max(1 - pos, 1e-6)
    W = torch.where(Y > 0.5, torch.tensor(wpos, device="cuda"), torch.tensor(wneg, device="cuda")).float()
    N = F.shape[0]
    Nrm = torch.from_numpy(norm).to("cuda")
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(N)).to("cuda")
        tot = 0.0
        nb = 0
        for i in range(0, N, batch):
            idx = order[i:i + batch]
            g, loss = sp.mlp_backward(P, F[idx].contiguous(), Y[idx].contiguous(), W[idx].contiguous(), Nrm)
            step += 1
            sp.mlp_adam(P, g, m, v, step, lr)
            tot += float(loss)
            nb += 1
        hist.append(tot / max(nb, 1))
        if ep % log_every == 0 or ep == epochs - 1:
            log(f"[train] epoch {ep} loss {hist[-1]:.4f}")
    return P.cpu().numpy(), norm, hist


def accuracy(params, norm, feat, label):
    p = sp.mlp_forward(torch.from_numpy(params).to("cuda"), torch.from_numpy(feat.astype(np.float32)).to("cuda"),
                       torch.from_numpy(norm).to("cuda")).cpu().numpy()
    pred = p >= 0.5
    y = label > 0.5
    tp = float(np.sum(pred & y))
    return dict(acc=float(np.mean(pred == y)), precision=tp / max(1.0, float(np.sum(pred))),
                recall=tp / max(1.0, float(np.sum(y))), positives=float(np.mean(y)))


def time_variant(h, which, b, reps=21):
    """Autotuned solve time: median of `reps` solves, each between HIP events
    on the current stream."""
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
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return float(np.median(ts)), x


def _geomean(r):
    return math.exp(float(np.mean(np.log(r))))


def choose_action(seeds, actions=ACTIONS):
    """(B, C) whose thin-level rewrite (levels with < B rows, budget B, cap C)
    is fastest in geometric mean against naive on the given matrices."""
    ratios = {a: [] for a in actions}
    for s in seeds:
        m = gen.policy_training_matrix(s)
        b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
        h = sp.Handle()
        h.analyze(*to_dev(m))
        h.rewrite(sp.THIN_ROWS, *NAIVE, 0)
        t_naive, _ = time_variant(h, sp.REWRITTEN, b)
        for a in actions:
            h.rewrite(sp.THIN_ROWS, float(a[0]), float(a[1]), 0)
            ratios[a].append(t_naive / time_variant(h, sp.REWRITTEN, b)[0])
        h.close()
        log(f"[action] seed {s}: " + " ".join(f"{a[0]},{a[1]:g}:{r[-1]:.3f}" for a, r in ratios.items()))
    score = {a: _geomean(r) for a, r in ratios.items()}
    best = max(actions, key=lambda a: score[a])
    log(f"[action] geomean naive/(B,C) rewrite: { {str(k): round(v, 4) for k, v in score.items()} } -> {best}")
    return best, score


def tier_grid(action):
    """Candidate (t_lo, t_hi) pairs; t_lo == t_hi leaves out the naive tier,
    t_hi above 1 leaves out the (B, C) tier."""
    his = (0.02, 0.1, 0.3, 0.5, 0.7, 0.9, 1.01)
    los = (0.02, 0.1, 0.3, 0.5)
    pairs = sorted({(lo, hi) for hi in his for lo in los + (hi,) if lo <= hi and lo <= 1.0})
    return [((lo, 0, 0.0), (hi, int(action[0]), float(action[1]))) for lo, hi in pairs]


def calibrate(params, norm, seeds, action):
    """Tier thresholds with the best geometric-mean time ratio naive / learned
    on the given matrices (each variant autotuned; ties: the higher
    thresholds, which rewrite less)."""
    grid = tier_grid(action)
    ratios = {g: [] for g in grid}
    pol = Policy(params, norm, list(grid[0]))
    for s in seeds:
        m = gen.policy_training_matrix(s)
        b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
        h = sp.Handle()
        h.analyze(*to_dev(m))
        h.rewrite(sp.THIN_ROWS, *NAIVE, 0)
        t_naive, _ = time_variant(h, sp.REWRITTEN, b)
        prob = pol.probs(h)
        for g in grid:
            mask, bud, cap = sp.mlp_actions(prob, list(g))
            h.rewrite(sp.THIN_ROWS, *NAIVE, 0, mask, level_budget=bud, level_fill_cap=cap)
            ratios[g].append(t_naive / time_variant(h, sp.REWRITTEN, b)[0])
        h.close()
        log(f"[calibrate] seed {s}: best pair so far x{max(r[-1] for r in ratios.values()):.3f}")
    score = {g: _geomean(r) for g, r in ratios.items()}
    best = max(sorted(grid, key=lambda g: (-g[1][0], -g[0][0])), key=lambda g: score[g])
    log("[calibrate] geomean naive/learned by (t_lo, t_hi): "
        + json.dumps({f"{g[0][0]},{g[1][0]}": round(v, 4) for g, v in score.items()}) + f" -> {best}")
    return list(best), score


def evaluate(policy: Policy, seeds, action, check=True):
    """Autotuned solve time of plain, naive, the constant (B, C) rule and
    learned on each seed. The rewritten solutions are checked against the
    plain solution (relative error <= 1e-10) and the plain one by its
    residual."""
    from paper_2206_05843_amd.policy import rewrite_learned
    out = []
    for s in seeds:
        m = gen.policy_training_matrix(s)
        b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
        xr = None
        res = {"seed": s, "n": m.n, "nnz": m.nnz}
        for name in ("plain", "naive", "constant", "learned"):
            h = sp.Handle()
            res_nlev = h.analyze(*to_dev(m))
            which = sp.ORIGINAL
            st = None
            if name == "naive":
                st = h.rewrite(sp.THIN_ROWS, *NAIVE, 0)
            elif name == "constant":
                st = h.rewrite(sp.THIN_ROWS, float(action[0]), float(action[1]), 0)
            elif name == "learned":
                st = rewrite_learned(h, policy, *NAIVE)
            if st is not None:
                res_nlev = st["nlev_after"]
                which = sp.REWRITTEN
            t, x = time_variant(h, which, b)
            h.check()
            if check:
                if xr is None:
                    xr = x.clone()
                    assert max(h.residual(b, x)) <= 1e-12 * (1.0 + float(x.abs().max())), (s, "residual")
                else:
                    err = float((x - xr).abs().max() / xr.abs().max())
                    assert err <= 1e-10, (s, name, err)
            res[name] = {"ms": t * 1e3, "nlev": res_nlev, "mode": h.get_schedule(which, 1)["mode"]}
            if st is not None:
                res[name].update(rows_rewritten=st["rows_rewritten"], nnz_Lp=st["nnz_Lp"], nnz_T=st["nnz_T"])
            h.close()
        for k in ("naive", "plain", "constant"):
            res[f"learned_vs_{k}"] = res[k]["ms"] / res["learned"]["ms"]
        log(f"[eval] seed {s} n={m.n} plain {res['plain']['ms']:.3f}ms naive {res['naive']['ms']:.3f}ms "
            f"constant {res['constant']['ms']:.3f}ms learned {res['learned']['ms']:.3f}ms "
            f"(x{res['learned_vs_naive']:.3f} vs naive)")
        out.append(res)
    g = {k: _geomean([r[f"learned_vs_{k}"] for r in out]) for k in ("naive", "plain", "constant")}
    return out, g


def evaluate_checkpoint(path, heldout, out):
    """The held-out comparison of a saved policy (its tiers and the action
    recorded with it) on seeds 2000 .. 2000 + heldout - 1, written to
    out/policy_eval.json."""
    pol = Policy.load(path)
    act = pol.meta.get("action", {})
    action = (int(act.get("budget", NAIVE[0])), float(act.get("fill_cap", NAIVE[1])))
    res, g = evaluate(pol, list(range(2000, 2000 + heldout)), action)
    summary = {"heldout_seeds": [2000, 2000 + heldout - 1], "tiers": [list(t) for t in pol.tiers],
               "geomean_learned_vs_naive": g["naive"], "geomean_learned_vs_plain": g["plain"],
               "geomean_learned_vs_constant": g["constant"], "per_matrix": res}
    with open(os.path.join(out, "policy_eval.json"), "w") as f:
        json.dump(summary, f, indent=1)
    log(f"[eval] geomean speedup learned vs naive {g['naive']:.4f}, vs plain {g['plain']:.4f}, "
        f"vs constant {g['constant']:.4f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--matrices", type=int, default=200)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--calib", type=int, default=10, help="validation matrices for the action and tiers (1900..)")
    ap.add_argument("--action", default="", help="B,C to skip the action search")
    ap.add_argument("--evaluate", default="", metavar="CKPT",
                    help="only measure the checkpoint CKPT (.npz with its .json) on the held-out seeds")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    if args.evaluate:
        evaluate_checkpoint(args.evaluate, args.heldout, args.out)
        return
    calib_seeds = list(range(1900, 1900 + max(args.calib, 1)))
    if args.action:
        bb, cc = args.action.split(",")
        action, action_score = (int(bb), float(cc)), {}
    else:
        action, action_score = choose_action(calib_seeds)
    seeds = list(range(args.first_seed, args.first_seed + args.matrices))
    feats, labels, deltas, owner = [], [], [], []
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=4) as ex:
        for i, m in enumerate(ex.map(gen.policy_training_matrix, seeds)):
            f, y, d, e = level_data(m, action)
            feats.append(f)
            labels.append(y)
            deltas.append(d)
            owner.append(np.full(len(y), i, np.int32))
            log(f"[data] {i + 1}/{len(seeds)} seed {seeds[i]} n={m.n} levels={len(y) + 1} emptied={int(e.sum())} "
                f"positive={int(y.sum())} ({time.perf_counter() - t0:.0f}s)")
    F = np.concatenate(feats)
    Y = np.concatenate(labels)
    D = np.concatenate(deltas)
    O = np.concatenate(owner)
    np.savez(os.path.join(args.out, "policy_data.npz"), feat=F, label=Y, delta=D, owner=O)
    val = O >= int(0.9 * len(seeds))
    params, norm, hist = train(F[~val], Y[~val], epochs=args.epochs)
    acc_tr = accuracy(params, norm, F[~val], Y[~val])
    acc_va = accuracy(params, norm, F[val], Y[val])
    log(f"[train] train {acc_tr} val {acc_va}")
    tiers, score = [(0.5, int(action[0]), float(action[1]))], {}
    if args.calib > 0:
        tiers, score = calibrate(params, norm, calib_seeds, action)
    meta = {"train_seeds": [seeds[0], seeds[-1]], "levels": int(F.shape[0]), "positive_rate": float(Y.mean()),
            "epochs": args.epochs, "loss_history": hist, "train_metrics": acc_tr, "val_metrics": acc_va,
            "action": {"budget": int(action[0]), "fill_cap": float(action[1]),
                       "geomean_naive_over_constant_by_action": {str(k): v for k, v in action_score.items()}},
            "label": "1 = emptied by the (budget, cap) rewrite and its rows cost less of the synchronisation-free "
                     "solve's critical path in L' than the level in L",
            "tiers": [list(t) for t in tiers], "calibration_seeds": [calib_seeds[0], calib_seeds[-1]],
            "calibration_geomean_naive_over_learned": {f"{g[0][0]},{g[1][0]}": v for g, v in score.items()}}
    pol = Policy(params, norm, tiers, meta)
    pol.save(os.path.join(args.out, "policy_ckpt.npz"))
    if args.heldout > 0:
        res, g = evaluate(pol, list(range(2000, 2000 + args.heldout)), action)
        summary = {"heldout_seeds": [2000, 2000 + args.heldout - 1], "tiers": [list(t) for t in tiers],
                   "geomean_learned_vs_naive": g["naive"], "geomean_learned_vs_plain": g["plain"],
                   "geomean_learned_vs_constant": g["constant"], "per_matrix": res}
        with open(os.path.join(args.out, "policy_eval.json"), "w") as f:
            json.dump(summary, f, indent=1)
        log(f"[eval] geomean speedup learned vs naive {g['naive']:.4f}, vs plain {g['plain']:.4f}, "
            f"vs constant {g['constant']:.4f}")


if __name__ == "__main__":
    main()
