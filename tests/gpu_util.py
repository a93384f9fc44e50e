"""Helpers of the GPU tests: run the library on a NumPy input, back to NumPy."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(G):
    import torch
    return torch.from_numpy(np.asfortranarray(G)).to("cuda:0")


def run_lib(ctx, G, p, check=False, **prm):
    from paper_1008_1371_amd import hsvd as H
    params = H.hsvd_default_params(**prm)
    R = H.hsvd_solve(ctx, to_dev(G), p, params, check=check)
    out = dict(status=R["status"], info=R["info"], sweeps=R["info"]["sweeps"])
    for k in ("sigma", "U", "V", "lam", "perm"):
        out[k] = R[k].cpu().numpy() if R[k] is not None else None
    return out
