"""Mixed-precision path (FP32 MFMA sweeps, FP64 J-re-orthogonalisation, FP64
refinement sweeps) vs the FP64 oracle (GPU).  The oracle has no FP32 phase:
parity is in the result, not the path."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import run_lib, say
from parity import compare, ordering_spread
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mixed(ctx, G, p, **kw):
    return run_lib(ctx, G, p, precision=1, **kw)


@pytest.mark.parametrize("n,p", [(3, 2), (40, 17), (128, 64), (200, 200), (256, 37)])
def test_mixed_gaussian(hsvd_ctx, n, p):
    G = W.gaussian(n, seed=300 + n)
    spread, ref = ordering_spread(G, p, block=32)
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0, res["status"]
    e = compare(res, ref, p)
    say("mixed", n, p, e, "fp32/fp64 sweeps", res["info"]["sweeps_fp32"], res["info"]["sweeps"],
        "ns", res["info"]["reorth_iters"], res["info"]["reorth_resid"], "ordering spread", spread)
    assert e["sigma_norm"] <= 1e-12
    gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
    assert e["U"] <= gate and e["V"] <= gate, e
    assert res["info"]["sweeps_fp32"] >= 1
    pins.check_invariants(G, p, res, tol=ref["tol"])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kappa,frac", [(1e2, 0.5), (1e6, 0.25), (1e10, 1.0)])
def test_mixed_graded512(hsvd_ctx, kappa, frac):
    n = 512
    p = int(n * frac)
    G = W.graded(n, kappa)
    spread, ref = ordering_spread(G, p, block=32)
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0
    e = compare(res, ref, p)
    say("mixed graded", kappa, p, e, "fp32/fp64", res["info"]["sweeps_fp32"], res["info"]["sweeps"],
        "ordering spread", spread)
    assert e["sigma_norm"] <= 1e-12
    gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
    assert e["U"] <= gate and e["V"] <= gate, e
    pins.check_invariants(G, p, res, tol=ref["tol"])


def test_mixed_no_v(hsvd_ctx):
    G = W.gaussian(192, seed=5)
    spread, ref = ordering_spread(G, 96, block=32)
    res = _mixed(hsvd_ctx, G, 96, want_v=0)
    assert res["status"] == 0 and res["V"] is None
    e = compare(res, ref, 96)
    assert e["sigma_norm"] <= 1e-12 and e["U"] <= max(1e-12, 10 * spread["U"]), (e, spread)


@pytest.mark.timeout(900)
def test_mixed_full_size_graded4096(hsvd_ctx):
    """n = 4096, kappa = 1e6, p = n/2: invariants and LAPACK eigenvalues."""
    G, p = W.workload("graded4096_k1e6_p0.5")
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0
    say("mixed 4096", {k: res["info"][k] for k in ("sweeps_fp32", "sweeps", "reorth_iters",
                                                   "reorth_resid", "ms_total")})
    pins.check_invariants(G, p, res, tol=1e-15 * 4096)


@pytest.mark.parametrize("mixed_pair", [False, True])
def test_mixed_orthogonal_columns(hsvd_ctx, mixed_pair):
    """Columns orthogonal to FP64 rounding, and the same with one pair of
    columns from different blocks mixed: the FP32 sweeps see these through the
    rounding of G to FP32, so whole launches of the inner solve are skipped
    while some pairs still rotate; the FP64 refinement then decides.  Result
    against the oracle."""
    n, p = 256, 100
    G = W.haar(n, seed=5) * np.logspace(0.0, -3.0, n)[None, :]
    if mixed_pair:
        G[:, [3, 70]] = G[:, [3, 70]] @ np.array([[1.0, 0.3], [0.2, 1.0]])
    spread, ref = ordering_spread(G, p, block=32)
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0, res["status"]
    e = compare(res, ref, p)
    say("mixed orthogonal columns", mixed_pair, e, "fp32/fp64 sweeps", res["info"]["sweeps_fp32"],
        res["info"]["sweeps"], "rotations", res["info"]["rotations"], "ordering spread", spread)
    assert e["sigma_norm"] <= 1e-12
    gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
    assert e["U"] <= gate and e["V"] <= gate, e
    pins.check_invariants(G, p, res, tol=ref["tol"])
