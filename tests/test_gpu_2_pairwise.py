"""Pairwise FP64 path vs the oracle on the same seeded inputs (GPU)."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import run_lib, say
from parity import compare, twin_spread
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gate(G, p, res, ref, *, uv_gate=1e-12, sigma_gate=1e-12):
    assert res["status"] == 0, res["status"]
    e = compare(res, ref, p)
    say("   errors", e, "sweeps lib/orc", res["info"]["sweeps"], ref["sweeps"])
    assert e["sigma_norm"] <= sigma_gate, e
    assert e["U"] <= uv_gate and e.get("V", 0.0) <= uv_gate, e
    pins.check_invariants(G, p, res, tol=ref["tol"])
    return e


@pytest.mark.parametrize("ordering", ["modmod", "roundrobin"])
def test_gauss128(hsvd_ctx, ordering):
    """128 x 128 N(0,1), p = 64, tol 1e-15 n."""
    G, p = W.workload("gauss128")
    say("gauss128", ordering)
    ref = oracle.hsvd(G, p, ordering=ordering)
    res = run_lib(hsvd_ctx, G, p, algo=1, ordering=0 if ordering == "modmod" else 1)
    _gate(G, p, res, ref)


@pytest.mark.parametrize("n,p", [(1, 1), (1, 0), (2, 1), (3, 1), (5, 5), (64, 0), (65, 32),
                                 (127, 100), (200, 7), (257, 128), (513, 256)])
def test_ragged_and_small(hsvd_ctx, n, p):
    G = W.colscaled(n, 2.0, seed=40 + n)
    say("ragged", n, p)
    ref = oracle.hsvd(G, p)
    res = run_lib(hsvd_ctx, G, p, algo=1)
    _gate(G, p, res, ref)


def test_unsorted_and_no_v(hsvd_ctx):
    G = W.gaussian(96, seed=5)
    ref = oracle.hsvd(G, 40, sort=False)
    res = run_lib(hsvd_ctx, G, 40, algo=1, sort=0)
    _gate(G, 40, res, ref)
    res2 = run_lib(hsvd_ctx, G, 40, algo=1, want_v=0)
    assert res2["status"] == 0 and res2["V"] is None
    e = compare(res2, ref, 40)
    assert e["sigma_norm"] <= 1e-12 and e["U"] <= 1e-12


@pytest.mark.timeout(900)
@pytest.mark.parametrize("p", [768, 1024])
def test_graded1024(hsvd_ctx, p):
    """Q1 diag(logspace(0, -8, 1024)) Q2, p = 768 and the definite case p = n.
    U and V are gated at 10x the spread of two oracle runs that differ only in
    summation order (the problem amplifies rounding by its conditioning)."""
    G = W.graded(1024, 1e8)
    say("graded1024", p)
    spread, ref = twin_spread(G, p, nthreads=0)
    say("   twin spread", spread)
    res = run_lib(hsvd_ctx, G, p, algo=1)
    gate = max(1e-12, 10 * max(spread["U"], spread.get("V", 0.0)))
    _gate(G, p, res, ref, uv_gate=gate)


def test_deterministic(hsvd_ctx):
    G = W.gaussian(200, seed=9)
    a = run_lib(hsvd_ctx, G, 77, algo=1)
    b = run_lib(hsvd_ctx, G, 77, algo=1)
    for k in ("sigma", "U", "V", "lam", "perm"):
        assert np.array_equal(a[k], b[k]), k


def test_error_paths(hsvd_ctx):
    from paper_1008_1371_amd import hsvd as H
    G = W.gaussian(16, seed=3)
    assert run_lib(hsvd_ctx, G, 8, algo=1, max_sweeps=1)["status"] == H.E_NOCONV
    Gd = G.copy()
    Gd[:, 12] = Gd[:, 3]
    assert run_lib(hsvd_ctx, Gd, 8, sort=0)["status"] == H.E_RANK
    Gz = G.copy()
    Gz[:, 5] = 0.0
    assert run_lib(hsvd_ctx, Gz, 8)["status"] == H.E_RANK
    Gn = G.copy()
    Gn[2, 2] = np.nan
    assert run_lib(hsvd_ctx, Gn, 8)["status"] == H.E_INVAL
    assert run_lib(hsvd_ctx, G, 17)["status"] == H.E_INVAL
    D = np.diag(np.arange(1.0, 17.0))
    R = run_lib(hsvd_ctx, D, 5)
    assert R["status"] == 0 and R["info"]["sweeps"] == 1 and R["info"]["rotations"] == 0
    assert np.array_equal(np.sort(R["sigma"]), np.arange(1.0, 17.0))


@pytest.mark.parametrize("n,algo,prec", [(96, 1, 0), (512, 2, 0), (512, 2, 1)])
def test_signature_in_any_order(hsvd_ctx, n, algo, prec):
    """hsvd_solve with J's signs scattered over the columns (jsig) equals hsvd_solve
    on the stably partitioned matrix, mapped back; invariants with that J.
    Pairwise, block and mixed paths."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    g = np.random.Generator(np.random.PCG64(n))
    G = W.gaussian(n, seed=70 + n)
    j = np.where(g.uniform(size=n) < 0.4, 1, -1).astype(np.int8)
    pi = np.r_[np.flatnonzero(j == 1), np.flatnonzero(j == -1)]
    p = int((j == 1).sum())
    prm = H.hsvd_default_params(algo=algo, precision=prec)
    Rj = H.hsvd_solve(hsvd_ctx, torch.from_numpy(G).cuda(), p, prm, jsig=torch.from_numpy(j).cuda())
    Rp = run_lib(hsvd_ctx, np.asfortranarray(G[:, pi]), p, algo=algo, precision=prec)
    sj, Uj, Vj = (Rj["sigma"].cpu().numpy(), Rj["U"].cpu().numpy(), Rj["V"].cpu().numpy())
    assert np.array_equal(sj[pi], Rp["sigma"])
    assert np.array_equal(Uj[:, pi], Rp["U"])
    assert np.array_equal(Vj[np.ix_(pi, pi)], Rp["V"])
    assert np.array_equal(Rj["lam"].cpu().numpy()[pi], Rp["lam"])
    assert np.array_equal(Rj["perm"].cpu().numpy(), pi[Rp["perm"]])
    J = np.diag(j.astype(float))
    assert np.linalg.norm(Vj.T @ J @ Vj - J) / np.linalg.norm(Vj, 2) ** 2 <= 1e-11
    assert np.linalg.norm(G @ Vj - Uj * sj) / np.linalg.norm(G) <= 1e-13 * np.linalg.norm(Vj, 2)
    assert ((Rj["lam"].cpu().numpy() > 0) == (j > 0)).all()


@pytest.mark.parametrize("ordering", [0, 1])
def test_pairwise_graph_replay_matches_eager(hsvd_ctx, ordering):
    """Each sweep replays one captured graph of the step launches, with the
    sort, reduction and read-back running eagerly in between: after every
    sweep (max_sweeps = 1 .. 4 returns that iterate) the state is bit-identical
    to launching the steps one by one."""
    G = W.graded(256, 1e6, seed1=71, seed2=72)
    for k in (1, 2, 3, 4):
        eager = run_lib(hsvd_ctx, G, 160, algo=1, ordering=ordering, graph=0, max_sweeps=k)
        graph = run_lib(hsvd_ctx, G, 160, algo=1, ordering=ordering, graph=1, max_sweeps=k)
        say("graph replay", ordering, k, eager["status"], graph["status"])
        assert eager["status"] == graph["status"]
        for key in ("sigma", "U", "V", "lam", "perm"):
            assert np.array_equal(eager[key], graph[key]), (k, key)
