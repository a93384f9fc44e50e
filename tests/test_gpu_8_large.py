"""The block path at n = 8192 (GPU): the largest order of the mixed-precision
workloads.  No oracle run at this size: the invariants, both precisions, and
the mixed result against the FP64 one."""
import numpy as np
import pytest

from gpu_util import check_invariants_gpu, say
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu


def _canon(R, p):
    import torch
    s = R["sigma"]
    idx = torch.arange(s.numel(), device=s.device)
    o = torch.cat([idx[:p][torch.argsort(-s[:p], stable=True)], idx[p:][torch.argsort(-s[p:], stable=True)]])
    return s[o], R["U"][:, o], R["V"][:, o]


@pytest.mark.timeout(900)
def test_colscaled8192_both_precisions(hsvd_ctx):
    """Column-scaled Gaussian n = 8192, p = 4096 (condition ~1e4), mixed and
    FP64.  Here every block pair's V update runs as one tile of the inner
    launch (128 block pairs, 128 free CUs)."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    G, p = W.workload("colscaled8192")
    n = G.shape[0]
    Gt = torch.from_numpy(G).cuda()
    tol = 1e-15 * n
    res = {}
    for prec in (1, 0):
        R = H.hsvd_solve(hsvd_ctx, Gt, p, H.hsvd_default_params(algo=2, precision=prec), check=False)
        i = R["info"]
        say("colscaled8192 precision", prec, "status", R["status"], "sweeps", i["sweeps_fp32"], i["sweeps"],
            "ms", i["ms_total"])
        assert R["status"] == 0
        check_invariants_gpu(Gt, p, R, tol=tol, sweeps=i["sweeps"] + i["sweeps_fp32"])
        res[prec] = R
    s1, U1, V1 = _canon(res[1], p)
    s0, U0, V0 = _canon(res[0], p)
    es = (torch.linalg.vector_norm(s1 - s0) / torch.linalg.vector_norm(s0)).item()
    rows = U0.abs().argmax(dim=0)
    cols = torch.arange(n, device=U0.device)
    flip = torch.sign(U0[rows, cols]) * torch.sign(U1[rows, cols])
    eu = (torch.linalg.matrix_norm(U1 * flip - U0) / torch.linalg.matrix_norm(U0)).item()
    ev = (torch.linalg.matrix_norm(V1 * flip - V0) / torch.linalg.matrix_norm(V0)).item()
    say("mixed vs fp64: sigma", es, "U", eu, "V", ev)
    assert es <= 1e-12
    # two converged iterates of different trajectories: U and V agree to the
    # level the stop rule leaves (off-diagonal up to tol = 8.2e-12 over the
    # relative gaps of the spectrum; 2.1e-9 measured), not to 1e-12
    assert eu <= 1e-7 and ev <= 1e-7, (eu, ev)


@pytest.mark.timeout(900)
def test_graded8192_both_precisions(hsvd_ctx):
    """Graded n = 8192 (Q1 diag(logspace(0, -6, n)) Q2, kappa = 1e6,
    p = n/2), mixed and FP64: the largest graded configuration of the
    mixed-precision workloads."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    G, p = W.workload("graded8192_k1e6_p0.5")
    n = G.shape[0]
    Gt = torch.from_numpy(G).cuda()
    tol = 1e-15 * n
    res = {}
    for prec in (1, 0):
        R = H.hsvd_solve(hsvd_ctx, Gt, p, H.hsvd_default_params(algo=2, precision=prec), check=False)
        i = R["info"]
        say("graded8192 precision", prec, "status", R["status"], "sweeps", i["sweeps_fp32"], i["sweeps"],
            "ms", i["ms_total"], "restart", i["fp64_restart"])
        assert R["status"] == 0
        check_invariants_gpu(Gt, p, R, tol=tol, sweeps=i["sweeps"] + i["sweeps_fp32"])
        res[prec] = R
    s1, U1, V1 = _canon(res[1], p)
    s0, U0, V0 = _canon(res[0], p)
    es = (torch.linalg.vector_norm(s1 - s0) / torch.linalg.vector_norm(s0)).item()
    rows = U0.abs().argmax(dim=0)
    cols = torch.arange(n, device=U0.device)
    flip = torch.sign(U0[rows, cols]) * torch.sign(U1[rows, cols])
    eu = (torch.linalg.matrix_norm(U1 * flip - U0) / torch.linalg.matrix_norm(U0)).item()
    ev = (torch.linalg.matrix_norm(V1 * flip - V0) / torch.linalg.matrix_norm(V0)).item()
    say("mixed vs fp64: sigma", es, "U", eu, "V", ev)
    # two converged iterates of different trajectories at tol = 8.2e-12: at
    # n = 4096 the oracle's own two orderings differ by 8.1e-13 in sigma on
    # this kind of matrix and by 1.2e-9 in U; gates at about 10x those
    assert es <= 1e-11, es
    assert eu <= 1e-7 and ev <= 1e-7, (eu, ev)


@pytest.mark.timeout(900)
def test_max_order(hsvd_ctx):
    """The largest order the library takes (bordered order r = 16384): a
    column-scaled Gaussian (condition ~1e4) of order n = 16384, p = n/2, on
    the mixed path, and the same matrix cut to n = 16383 (one border column)
    on the FP64 block path, both against the invariants; one order more is
    rejected before any launch."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    n = 16384
    G = W.colscaled(n, 4.0, seed=16384)
    for prec, m in ((1, n), (0, n - 1)):
        Gt = torch.from_numpy(G[:m, :m]).cuda()
        p = m // 2
        say("max order: n", m, "p", p, "precision", prec)
        R = H.hsvd_solve(hsvd_ctx, Gt, p, H.hsvd_default_params(algo=2, precision=prec), check=False)
        i = R["info"]
        say("   status", R["status"], "sweeps", i["sweeps_fp32"], i["sweeps"], "ms", i["ms_total"])
        assert R["status"] == 0
        check_invariants_gpu(Gt, p, R, tol=1e-15 * m, sweeps=i["sweeps"] + i["sweeps_fp32"])
        del Gt, R
        torch.cuda.empty_cache()
    big = torch.zeros((n + 1, n + 1), dtype=torch.float64, device="cuda")
    big.diagonal().fill_(1.0)
    for algo in (1, 2):
        R = H.hsvd_solve(hsvd_ctx, big, (n + 1) // 2, H.hsvd_default_params(algo=algo), check=False)
        assert R["status"] == H.E_INVAL, (algo, R["status"])
