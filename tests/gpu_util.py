"""Helpers shared by the GPU tests: move generator matrices to the device."""
import numpy as np
import torch


def dev(m):
    d = torch.device("cuda")
    return (torch.from_numpy(np.ascontiguousarray(m.row_ptr)).to(d), torch.from_numpy(np.ascontiguousarray(m.col)).to(d),
            torch.from_numpy(np.ascontiguousarray(m.val)).to(d))


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")
