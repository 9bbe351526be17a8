"""Train and evaluate the learned rewrite policy on the GPU.

    python -m paper_2206_05843_amd.train_policy --out DIR [--matrices 200] [--heldout 20]

Data. For each seeded power-law training matrix (n ~ U[50k, 500k]) the
library measures, on the device, the time of every level of one solve of L
and of one solve of L' after the naive rewrite (levels with < 32 rows, fill
cap 4x), with every level inside one workgroup (sptrsv_level_times). A level
that the naive rewrite empties is labelled 1 when the time its rows cost in
their new levels of L' (their share, by row entries, of those levels' times)
is below the time the level took in L, else 0; levels that are not emptied are
labelled 0. The features are the 20 per-level features of the original levels
(sptrsv_level_features), the row constraints of Sec. III.A among them.

Training. Mean class-balanced binary cross-entropy, Adam, minibatches; forward,
backward and the Adam step are the library's kernels. Features are
standardised with the training set's mean and standard deviation, which are
stored in the checkpoint with the weights.

Calibration. The decision threshold on the network's probability is chosen
on separate validation matrices (seeds 1900..): the one with the best
geometric-mean solve-time ratio against the naive rewrite (ties: the higher
threshold, which rewrites less).

Evaluation. On held-out seeds, plain, naive and learned are autotuned and
timed; the rewritten solutions are checked against the plain solution
(relative error <= 1e-10) and the plain one by its residual.
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


def log(*a):
    print(*a, flush=True)


def to_dev(m):
    d = torch.device("cuda")
    return (torch.from_numpy(m.row_ptr).to(d), torch.from_numpy(m.col).to(d), torch.from_numpy(m.val).to(d))


def level_data(m, reps: int = 3):
    """Features, labels and time deltas of the original levels of m."""
    h = sp.Handle()
    h.analyze(*to_dev(m))
    feat = h.level_features().cpu().numpy()
    b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
    t_plain = np.mean([h.level_times(b, sp.ORIGINAL).cpu().numpy() for _ in range(reps)], axis=0)
    h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
    t_rew = np.mean([h.level_times(b, sp.REWRITTEN).cpu().numpy() for _ in range(reps)], axis=0)
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


def time_variant(h, which, b, reps=20):
    h.autotune(which, 1)
    x = torch.empty_like(b)
    for _ in range(3):
        h.solve(b, which, x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        h.solve(b, which, x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, x


def calibrate(params, norm, seeds, thresholds=(0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.99)):
    """Threshold with the best geometric-mean time ratio naive / learned on
    the given matrices (each variant autotuned)."""
    ratios = {t: [] for t in thresholds}
    for s in seeds:
        m = gen.policy_training_matrix(s)
        b = torch.from_numpy(gen.rhs(m, 1)[0]).to("cuda")
        h = sp.Handle()
        h.analyze(*to_dev(m))
        h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)
        t_naive, _ = time_variant(h, sp.REWRITTEN, b)
        for t in thresholds:
            pol = Policy(params, norm, t)
            h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0, pol.mask_for(h))
            t_l, _ = time_variant(h, sp.REWRITTEN, b)
            ratios[t].append(t_naive / t_l)
        h.close()
    score = {t: math.exp(np.mean(np.log(r))) for t, r in ratios.items()}
    best = max(sorted(thresholds, reverse=True), key=lambda t: score[t])
    log(f"[calibrate] geomean naive/learned by threshold: {json.dumps({str(k): round(v, 4) for k, v in score.items()})}"
        f" -> {best}")
    return best, score


def evaluate(policy: Policy, seeds, check=True):
    """Autotuned solve time of plain, naive and learned on each seed. The
    rewritten solutions are checked against the plain solution (relative error
    <= 1e-10) and the plain one by its residual."""
    out = []
    for s in seeds:
        m = gen.policy_training_matrix(s)
        b_np = gen.rhs(m, 1)
        b = torch.from_numpy(b_np[0]).to("cuda")
        xr = None
        res = {"seed": s, "n": m.n}
        for name in ("plain", "naive", "learned"):
            h = sp.Handle()
            res_nlev = h.analyze(*to_dev(m))
            which = sp.ORIGINAL
            if name == "naive":
                res_nlev = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0)["nlev_after"]
                which = sp.REWRITTEN
            elif name == "learned":
                res_nlev = h.rewrite(sp.THIN_ROWS, 32.0, 4.0, 0, policy.mask_for(h))["nlev_after"]
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
            res[name] = {"ms": t * 1e3, "nlev": res_nlev}
            h.close()
        res["learned_vs_naive"] = res["naive"]["ms"] / res["learned"]["ms"]
        res["learned_vs_plain"] = res["plain"]["ms"] / res["learned"]["ms"]
        log(f"[eval] seed {s} n={m.n} plain {res['plain']['ms']:.3f}ms naive {res['naive']['ms']:.3f}ms "
            f"learned {res['learned']['ms']:.3f}ms (x{res['learned_vs_naive']:.3f} vs naive)")
        out.append(res)
    g = math.exp(np.mean([math.log(r["learned_vs_naive"]) for r in out]))
    gp = math.exp(np.mean([math.log(r["learned_vs_plain"]) for r in out]))
    return out, g, gp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--matrices", type=int, default=200)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--heldout", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--calib", type=int, default=10, help="validation matrices for the threshold (seeds 1900..)")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    seeds = list(range(args.first_seed, args.first_seed + args.matrices))
    feats, labels, deltas, owner = [], [], [], []
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=4) as ex:
        for i, m in enumerate(ex.map(gen.policy_training_matrix, seeds)):
            f, y, d, e = level_data(m)
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
    thr, score = (0.5, {})
    if args.calib > 0:
        thr, score = calibrate(params, norm, list(range(1900, 1900 + args.calib)))
    meta = {"train_seeds": [seeds[0], seeds[-1]], "levels": int(F.shape[0]), "positive_rate": float(Y.mean()),
            "epochs": args.epochs, "loss_history": hist, "train_metrics": acc_tr, "val_metrics": acc_va,
            "label": "1 = emptied by the naive rewrite and its rows cost less time in L' than the level in L",
            "threshold": thr, "calibration_seeds": [1900, 1900 + args.calib - 1] if args.calib > 0 else [],
            "calibration_geomean_naive_over_learned": {str(k): v for k, v in score.items()}}
    pol = Policy(params, norm, thr, meta)
    pol.save(os.path.join(args.out, "policy_ckpt.npz"))
    if args.heldout > 0:
        res, g, gp = evaluate(pol, list(range(2000, 2000 + args.heldout)))
        summary = {"heldout_seeds": [2000, 2000 + args.heldout - 1], "geomean_learned_vs_naive": g,
                   "geomean_learned_vs_plain": gp, "per_matrix": res}
        with open(os.path.join(args.out, "policy_eval.json"), "w") as f:
            json.dump(summary, f, indent=1)
        log(f"[eval] geomean speedup learned vs naive {g:.4f}, vs plain {gp:.4f}")


if __name__ == "__main__":
    main()
