"""Learned rewrite policy: which levels to rewrite, and how far.

The paper's naive strategy rewrites every thin level under one target budget
and fill cap (Sec. III) and notes that a rewrite is not always worth its cost
(Sec. III.A). Here a small network over per-level features gives each level a
probability that rewriting it pays, and tiers map that probability to an
action: below the first tier's threshold the level is not a source; in tier j
it is a source whose rows may fill a target up to budget_j rows with at most
cap_j times their own entries (0 = the rewrite's own budget and cap). So the
policy can move rows naive cannot (a larger budget or cap on the levels the
network trusts) and keep rows naive would move. The stop-and-retarget logic
of the scan stays in force; a missing or unusable checkpoint falls back to the
thin-level test.

Inference is on the device: sptrsv_level_features -> sptrsv_mlp_forward ->
sptrsv_mlp_actions (mask, per-level budget and cap handed to sptrsv_rewrite).
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import sptrsv as _sp

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CKPT = os.path.join(HERE, "policy_ckpt.npz")


def _tiers(tiers):
    """[(threshold, budget, cap), ...] with ascending thresholds; a bare number
    is one tier at that threshold with the rewrite's own budget and cap."""
    if isinstance(tiers, (int, float, np.floating)):
        tiers = [(float(tiers), 0, 0.0)]
    out = [(float(t), int(b), float(c)) for t, b, c in tiers]
    if not 1 <= len(out) <= _sp.MAX_TIERS:
        raise ValueError("a policy has 1 to 4 tiers")
    if any(out[i][0] > out[i + 1][0] for i in range(len(out) - 1)) or any(b < 0 or c < 0 for _, b, c in out):
        raise ValueError("tiers need ascending thresholds and budgets, caps >= 0")
    return out


class Policy:
    def __init__(self, params: np.ndarray, norm: np.ndarray, tiers=0.5, meta: dict | None = None):
        params = np.asarray(params, np.float32).reshape(-1)
        norm = np.asarray(norm, np.float32).reshape(-1)
        if params.size != _sp.MLP_NPARAM or norm.size != 2 * _sp.MLP_NIN:
            raise ValueError("bad policy checkpoint shape")
        if not (np.all(np.isfinite(params)) and np.all(np.isfinite(norm))):
            raise ValueError("non-finite policy checkpoint")
        self.params = torch.from_numpy(params).to("cuda")
        self.norm = torch.from_numpy(norm).to("cuda")
        self.tiers = _tiers(tiers)
        self.meta = meta or {}

    @property
    def threshold(self) -> float:
        """The lowest threshold: levels below it are not sources."""
        return self.tiers[0][0]

    def probs(self, h: _sp.Handle):
        return _sp.mlp_forward(self.params, h.level_features(), self.norm)

    def actions(self, h: _sp.Handle, prob=None):
        """(mask, budget, cap) device arrays over the ORIGINAL levels of h
        (level 0 never a source)."""
        return _sp.mlp_actions(self.probs(h) if prob is None else prob, self.tiers)

    def mask_for(self, h: _sp.Handle):
        """uint8 device mask over the ORIGINAL levels of h (level 0 never a source)."""
        return self.actions(h)[0]

    def save(self, path: str = DEFAULT_CKPT):
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(),
                 tiers=np.array(self.tiers, np.float64).reshape(-1, 3))
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(self.meta, f, indent=1)

    @staticmethod
    def load(path: str = DEFAULT_CKPT) -> "Policy":
        with np.load(path, allow_pickle=False) as z:
            params, norm = z["params"], z["norm"]
            if "tiers" in z:
                tiers = [(float(t), int(b), float(c)) for t, b, c in np.asarray(z["tiers"]).reshape(-1, 3)]
            else:
                tiers = float(z["threshold"][0])
        meta = {}
        jp = os.path.splitext(path)[0] + ".json"
        if os.path.exists(jp):
            with open(jp) as f:
                meta = json.load(f)
        return Policy(params, norm, tiers, meta)


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights and zero biases in the flat layout of the C ABI
    (W1[64,20] b1[64] W2[64,64] b2[64] W3[64] b3[1])."""
    rng = np.random.default_rng(seed)
    parts = []
    nin = _sp.MLP_NIN
    for shape, fan_in in [((64, nin), nin), ((64,), 0), ((64, 64), 64), ((64,), 0), ((64,), 64), ((1,), 0)]:
        if fan_in:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


def load_default() -> Policy | None:
    """The committed checkpoint, or None (callers then use the thin-level test)."""
    try:
        return Policy.load(DEFAULT_CKPT)
    except (OSError, KeyError, ValueError):
        return None


def rewrite_learned(h: _sp.Handle, policy: Policy | None, thin_threshold=32.0, fill_cap=4.0, max_distance=0,
                    max_indegree=0, max_spread=0, critical_only=False):
    """Rewrite with the policy's per-level actions (fallback: the thin-level
    test with thin_threshold and fill_cap). A tier's budget and cap of 0 take
    thin_threshold and fill_cap. The row constraints of Sec. III.A (indegree <
    max_indegree, column span < max_spread, longest-path rows only) apply to
    each row of the chosen levels, as in the plain strategies; 0 / False
    leaves them off."""
    if policy is None:
        return h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, max_distance, None, max_indegree=max_indegree,
                         max_spread=max_spread, critical_only=critical_only)
    mask, budget, cap = policy.actions(h)
    return h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, max_distance, mask, max_indegree=max_indegree,
                     max_spread=max_spread, critical_only=critical_only, level_budget=budget, level_fill_cap=cap)


def rewrite_learned_checked(h: _sp.Handle, policy: Policy | None, nrhs: int = 1, thin_threshold=32.0, fill_cap=4.0,
                            csr=None, **knobs):
    """The learned rewrite with a measured per-matrix fallback: the policy's
    rewrite and the naive rule's (thin_threshold, fill_cap) are each
    autotuned for nrhs right-hand sides on this matrix, and h keeps the
    faster one (ties: the learned one), autotuned. With csr = (row_ptr, col,
    val) of the matrix h analysed, the naive rewrite is timed on a scratch
    handle, so h is rewritten again only when naive wins. Returns (stats,
    chosen) with chosen in {"learned", "naive"}."""
    if policy is None:
        st = h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, **knobs)
        h.autotune(_sp.REWRITTEN, nrhs)
        return st, "naive"
    st_l = rewrite_learned(h, policy, thin_threshold, fill_cap, **knobs)
    t_learned = h.autotune(_sp.REWRITTEN, nrhs)
    if csr is not None:
        g = _sp.Handle()
        try:
            g.analyze(*csr)
            g.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, **knobs)
            t_naive = g.autotune(_sp.REWRITTEN, nrhs)
        finally:
            g.close()
        if t_naive >= t_learned:
            return st_l, "learned"
        st = h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, **knobs)
        h.autotune(_sp.REWRITTEN, nrhs)
        return st, "naive"
    st = h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, **knobs)
    t_naive = h.autotune(_sp.REWRITTEN, nrhs)
    if t_naive < t_learned:
        return st, "naive"
    st = rewrite_learned(h, policy, thin_threshold, fill_cap, **knobs)
    h.autotune(_sp.REWRITTEN, nrhs)
    return st, "learned"
