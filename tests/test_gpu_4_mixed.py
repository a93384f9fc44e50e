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


def _gate(res, ref, p, spread, n):
    """sigma normwise to 1e-12; sigma componentwise, U and V to 10x the
    oracle's ordering spread (at least 1e-12); the J-re-orthogonalisation
    accepted without a restart."""
    e = compare(res, ref, p)
    assert e["sigma_norm"] <= 1e-12, e
    assert e["sigma_max"] <= max(1e-12, 10 * spread["sigma_max"]), (e, spread)
    gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
    assert e["U"] <= gate and e["V"] <= gate, (e, spread)
    assert res["info"]["fp64_restart"] == 0
    assert res["info"]["reorth_resid"] <= 16384 * n * 2.0 ** -53, res["info"]["reorth_resid"]
    return e


@pytest.mark.parametrize("n,p", [(3, 2), (40, 17), (128, 64), (200, 200), (256, 37)])
def test_mixed_gaussian(hsvd_ctx, n, p):
    G = W.gaussian(n, seed=300 + n)
    spread, ref = ordering_spread(G, p, block=32)
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0, res["status"]
    say("mixed", n, p, compare(res, ref, p), "fp32/fp64 sweeps", res["info"]["sweeps_fp32"],
        res["info"]["sweeps"], "ns", res["info"]["reorth_iters"], res["info"]["reorth_resid"],
        "ordering spread", spread)
    _gate(res, ref, p, spread, n)
    assert res["info"]["sweeps_fp32"] >= 1
    pins.check_invariants(G, p, res, tol=ref["tol"])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kappa,frac", [(1e2, 0.5), (1e6, 0.25), (1e10, 0.25), (1e10, 0.5), (1e10, 1.0)])
def test_mixed_graded512(hsvd_ctx, kappa, frac):
    """The graded inputs of the mixed-precision workloads at n = 512, the
    indefinite kappa = 1e10 cases included."""
    n = 512
    p = int(n * frac)
    G = W.graded(n, kappa)
    spread, ref = ordering_spread(G, p, block=32)
    res = _mixed(hsvd_ctx, G, p)
    assert res["status"] == 0
    say("mixed graded", kappa, p, compare(res, ref, p), "fp32/fp64", res["info"]["sweeps_fp32"],
        res["info"]["sweeps"], "ns", res["info"]["reorth_iters"], res["info"]["reorth_resid"],
        "ordering spread", spread)
    _gate(res, ref, p, spread, n)
    pins.check_invariants(G, p, res, tol=ref["tol"])


def test_mixed_no_v(hsvd_ctx):
    G = W.gaussian(192, seed=5)
    spread, ref = ordering_spread(G, 96, block=32)
    res = _mixed(hsvd_ctx, G, 96, want_v=0)
    assert res["status"] == 0 and res["V"] is None
    e = compare(res, ref, 96)
    assert e["sigma_norm"] <= 1e-12 and e["U"] <= max(1e-12, 10 * spread["U"]), (e, spread)
    assert e["sigma_max"] <= max(1e-12, 10 * spread["sigma_max"]), (e, spread)


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
    say("mixed orthogonal columns", mixed_pair, compare(res, ref, p), "fp32/fp64 sweeps",
        res["info"]["sweeps_fp32"], res["info"]["sweeps"], "rotations", res["info"]["rotations"],
        "ordering spread", spread)
    _gate(res, ref, p, spread, n)
    pins.check_invariants(G, p, res, tol=ref["tol"])


@pytest.mark.parametrize("n,p", [(128, 64), (300, 100)])
def test_mixed_forced_restart_equals_fp64(hsvd_ctx, n, p):
    """An accepted re-orthogonalisation residual below anything reachable
    forces the FP64 restart from G: the result is then bit-identical to the
    plain FP64 block solve (same launches from the set-up on)."""
    G = W.colscaled(n, 3.0, seed=400 + n)
    res = _mixed(hsvd_ctx, G, p, reorth_accept=1e-300)
    f64 = run_lib(hsvd_ctx, G, p, algo=2)
    say("forced restart", n, p, res["status"], res["info"]["fp64_restart"], res["info"]["sweeps_fp32"],
        res["info"]["sweeps"], f64["info"]["sweeps"])
    assert res["status"] == 0 and res["info"]["fp64_restart"] == 1 and res["info"]["sweeps_fp32"] >= 1
    assert res["info"]["sweeps"] == f64["info"]["sweeps"]
    for key in ("sigma", "U", "V", "lam", "perm"):
        assert np.array_equal(res[key], f64[key]), key


def test_mixed_near_parallel_hyperbolic_pair(hsvd_ctx):
    """Two columns of opposite sign that are parallel to about 1e-4: the FP32
    Gram cannot resolve a_ii + a_jj - 2|a_ij| (relative size 1e-8) and its
    sweeps may flag the pair as rank deficient; FP64 resolves it.  The mixed
    solve must still succeed (restarting in FP64 if its FP32 phase flags the
    pair) and match the oracle."""
    n, p = 128, 64
    g = np.random.Generator(np.random.PCG64(41))
    G = np.asfortranarray(g.standard_normal((n, n)))
    G[:, 100] = G[:, 10] * (1.0 + 1e-4) + 1e-4 * g.standard_normal(n) / np.sqrt(n) * np.linalg.norm(G[:, 10])
    spread, ref = ordering_spread(G, p, block=32)
    assert ref["status"] == 0, ref["status"]
    res = _mixed(hsvd_ctx, G, p)
    say("near-parallel hyperbolic pair: status", res["status"], "restart", res["info"]["fp64_restart"],
        "sweeps", res["info"]["sweeps_fp32"], res["info"]["sweeps"], compare(res, ref, p), "spread", spread)
    assert res["status"] == 0
    e = compare(res, ref, p)
    assert e["sigma_norm"] <= 1e-12, e
    gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
    assert e["U"] <= gate and e["V"] <= gate, (e, spread)
