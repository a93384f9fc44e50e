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


def spectral_norm_gpu(A, iters=30):
    """||A||_2 by power iteration on A^T A (seeded start), on the GPU."""
    import torch
    g = torch.Generator(device=A.device).manual_seed(1)
    x = torch.randn(A.shape[1], dtype=A.dtype, device=A.device, generator=g)
    for _ in range(iters):
        x = A.t() @ (A @ x)
        x = x / torch.linalg.vector_norm(x)
    return torch.linalg.vector_norm(A @ x).item()


def check_invariants_gpu(Gt, p, R, *, tol, sweeps):
    """The invariants of pins.check_invariants that stay cheap at large n
    (U^T U, V^T J V, G V = U Sigma, lambda = sigma^2 j), with the same bounds,
    computed with FP64 torch products on the GPU; no eigensolver."""
    import torch
    U64 = np.finfo(np.float64).eps / 2
    n = Gt.shape[0]
    U, s, V, lam = R["U"], R["sigma"], R["V"], R["lam"]
    j = torch.ones(n, dtype=torch.float64, device=Gt.device)
    j[p:] = -1.0
    UtU = U.t() @ U
    d = torch.diagonal(UtU)
    off = (UtU - torch.diag(d)).abs().max().item()
    assert off <= 2 * tol, ("U^T U off-diagonal", off, tol)
    assert (d - 1).abs().max().item() <= 8 * n * U64
    if V is not None:
        vn = spectral_norm_gpu(V) ** 2
        bound = 4 * n * np.sqrt(n * max(sweeps, 1)) * U64
        r1 = (torch.linalg.matrix_norm(V.t() @ (V * j[:, None]) - torch.diag(j)) / vn).item()
        assert r1 <= bound, ("V^T J V", r1, bound)
        r2 = (torch.linalg.matrix_norm(Gt @ V - U * s[None, :]) /
              (torch.linalg.matrix_norm(Gt) * max(1.0, vn ** 0.5))).item()
        assert r2 <= 10 * np.sqrt(n) * U64, ("G V - U S", r2)
    assert bool(((lam > 0) == (torch.arange(n, device=lam.device) < p)).all())
    assert bool(((lam.abs() - s * s).abs() <= 4 * np.finfo(np.float64).eps * s * s).all())
    return off
