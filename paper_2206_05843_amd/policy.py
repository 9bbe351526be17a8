"""Learned rewrite policy: which levels to rewrite.

The paper's naive strategy rewrites every thin level (Sec. III) and discusses
that a rewrite is not always worth its cost (Sec. III.A). This policy replaces
the thin-level test with a small network over per-level features; the
strategy's budget, fill cap and stop-and-retarget logic stay in force, and a
missing or unusable checkpoint falls back to the thin-level test.

Inference is on the device: sptrsv_level_features -> sptrsv_mlp_forward ->
sptrsv_mlp_mask (the level mask handed to sptrsv_rewrite).
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import sptrsv as _sp

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CKPT = os.path.join(HERE, "policy_ckpt.npz")


class Policy:
    def __init__(self, params: np.ndarray, norm: np.ndarray, threshold: float = 0.5, meta: dict | None = None):
        params = np.asarray(params, np.float32).reshape(-1)
        norm = np.asarray(norm, np.float32).reshape(-1)
        if params.size != _sp.MLP_NPARAM or norm.size != 2 * _sp.MLP_NIN:
            raise ValueError("bad policy checkpoint shape")
        if not (np.all(np.isfinite(params)) and np.all(np.isfinite(norm))):
            raise ValueError("non-finite policy checkpoint")
        self.params = torch.from_numpy(params).to("cuda")
        self.norm = torch.from_numpy(norm).to("cuda")
        self.threshold = float(threshold)
        self.meta = meta or {}

    def probs(self, h: _sp.Handle):
        return _sp.mlp_forward(self.params, h.level_features(), self.norm)

    def mask_for(self, h: _sp.Handle):
        """uint8 device mask over the ORIGINAL levels of h (level 0 never a source)."""
        return _sp.mlp_mask(self.probs(h), self.threshold)

    def save(self, path: str = DEFAULT_CKPT):
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(),
                 threshold=np.array([self.threshold], np.float32))
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(self.meta, f, indent=1)

    @staticmethod
    def load(path: str = DEFAULT_CKPT) -> "Policy":
        with np.load(path, allow_pickle=False) as z:
            params, norm, thr = z["params"], z["norm"], float(z["threshold"][0])
        meta = {}
        jp = os.path.splitext(path)[0] + ".json"
        if os.path.exists(jp):
            with open(jp) as f:
                meta = json.load(f)
        return Policy(params, norm, thr, meta)


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
    """Rewrite with the policy's level mask (fallback: the thin-level test).
    The row constraints of Sec. III.A (indegree < max_indegree, column span <
    max_spread, longest-path rows only) apply to each row of the chosen levels,
    as in the plain strategies; 0 / False leaves them off."""
    mask = policy.mask_for(h) if policy is not None else None
    return h.rewrite(_sp.THIN_ROWS, thin_threshold, fill_cap, max_distance, mask, max_indegree=max_indegree,
                     max_spread=max_spread, critical_only=critical_only)
