"""Batched solver: many independent problems of uneven order and signature (GPU)."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import say
from parity import compare, twin_spread
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(ctx, ns, ps, Gs, **prm):
    import torch

    from paper_1008_1371_amd import hsvd as H
    flat, offs = W.pack_batch(Gs)
    voffs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    R = H.hsvd_solve_batched(ctx, ns, ps, torch.from_numpy(flat).cuda(), offs, voffs,
                             H.hsvd_default_params(**prm), check=False)
    out = []
    sig, lam = R["sigma"].cpu().numpy(), R["lam"].cpu().numpy()
    U = R["U"].cpu().numpy()
    V = R["V"].cpu().numpy() if R["V"] is not None else None
    for k, n in enumerate(ns):
        o, v = offs[k], voffs[k]
        out.append(dict(status=int(R["statuses"][k]), sweeps=int(R["sweeps"][k]), info=R["infos"][k],
                        sigma=sig[v:v + n], lam=lam[v:v + n],
                        U=U[o:o + n * n].reshape(n, n, order="F"),
                        V=V[o:o + n * n].reshape(n, n, order="F") if V is not None else None,
                        perm=np.argsort(-sig[v:v + n])))
    return R, out


def test_batched_small_vs_oracle(hsvd_ctx):
    ns, ps, Gs = W.batch(40, seed_sizes=77, seed_g=9000)
    say("batched", list(ns))
    R, res = _run(hsvd_ctx, ns, ps, Gs)
    assert R["status"] == 0, R["statuses"]
    for k, (n, p, G) in enumerate(zip(ns, ps, Gs)):
        spread, ref = twin_spread(G, int(p), block=32)
        e = compare(res[k], ref, int(p))
        gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
        assert e["sigma_norm"] <= 1e-12 and e["U"] <= gate and e["V"] <= gate, (k, n, p, e, spread)
        assert res[k]["sweeps"] == ref["sweeps"] or abs(res[k]["sweeps"] - ref["sweeps"]) <= 1
        r = dict(res[k])
        r["sweeps"] = res[k]["sweeps"]
        pins.check_invariants(G, int(p), r, tol=1e-15 * n)


def test_batched_edge_cases(hsvd_ctx):
    """n = 1, definite (p = 0, p = n), a duplicate-column problem (rank
    failure stays local to its problem) and max_sweeps = 1."""
    g = np.random.Generator(np.random.PCG64(4))
    Gs = [g.standard_normal((n, n)) for n in (1, 5, 64, 65, 130)]
    ns = np.array([1, 5, 64, 65, 130], np.int32)
    ps = np.array([1, 0, 64, 30, 65], np.int32)
    R, res = _run(hsvd_ctx, ns, ps, Gs)
    assert R["status"] == 0, R["statuses"]
    for k in range(len(ns)):
        ref = oracle.hsvd(Gs[k], int(ps[k]), block=32)
        assert compare(res[k], ref, int(ps[k]))["sigma_norm"] <= 1e-12
    Gz = [G.copy() for G in Gs]
    Gz[3][:, 7] = 0.0
    R, res = _run(hsvd_ctx, ns, ps, Gz)
    st = R["statuses"]
    assert st[3] == -3 and all(st[k] == 0 for k in (0, 1, 2, 4)), st
    R, res = _run(hsvd_ctx, ns, ps, Gs, max_sweeps=1)
    assert (R["statuses"][2:] == -2).all(), R["statuses"]


@pytest.mark.timeout(900)
def test_batched_full_size(hsvd_ctx):
    """10,000 problems, n ~ U{8..256}, p ~ U{0..n}: every problem converges;
    invariants on a sample; the oracle on sampled problems one by one."""
    ns, ps, Gs = W.batch(10000)
    R, res = _run(hsvd_ctx, ns, ps, Gs)
    say("batched 10k", "max sweeps", int(R["sweeps"].max()), "rotations",
        sum(i["rotations"] for i in R["infos"]), "ms", R["infos"][0]["ms_total"])
    assert R["status"] == 0 and (R["statuses"] == 0).all()
    g = np.random.Generator(np.random.PCG64(11))
    for k in g.choice(len(ns), 24, replace=False):
        pins.check_invariants(Gs[k], int(ps[k]), res[k], tol=1e-15 * ns[k])
    for k in g.choice(len(ns), 6, replace=False):
        spread, ref = twin_spread(Gs[k], int(ps[k]), block=32)
        e = compare(res[k], ref, int(ps[k]))
        gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
        assert e["sigma_norm"] <= 1e-12 and e["U"] <= gate and e["V"] <= gate, (k, e, spread)


def test_batched_graph_replay_matches_eager(hsvd_ctx):
    """Each group's sweep captured once as a HIP graph and replayed gives
    bit-identical results to eager launches; graph runs before and after an
    eager run (and the eager single-problem solver in between) agree."""
    ns, ps, Gs = W.batch(24, seed_sizes=91, seed_g=9100)
    R1, a = _run(hsvd_ctx, ns, ps, Gs, graph=1)
    R2, b = _run(hsvd_ctx, ns, ps, Gs, graph=0)
    from gpu_util import run_lib
    run_lib(hsvd_ctx, Gs[0], int(ps[0]))
    R3, c = _run(hsvd_ctx, ns, ps, Gs, graph=1)
    assert R1["status"] == R2["status"] == R3["status"] == 0
    for k in range(len(ns)):
        for key in ("sigma", "U", "V", "lam"):
            assert np.array_equal(a[k][key], b[k][key]), (k, key)
            assert np.array_equal(a[k][key], c[k][key]), (k, key)
        assert a[k]["sweeps"] == b[k]["sweeps"] == c[k]["sweeps"]


def test_batched_mixed_vs_oracle(hsvd_ctx):
    """Mixed precision over a batch: FP32 block sweeps (each problem leaving
    them by its own switch rule), the batched J-re-orthogonalisation, FP64
    refinement.  Each problem against the FP64 oracle: sigma to 1e-12, U and V
    to 10x the ordering spread (the mixed trajectory is its own)."""
    from parity import ordering_spread
    ns, ps, Gs = W.batch(30, lo=8, hi=200, seed_sizes=78, seed_g=9100)
    say("batched mixed", list(ns))
    R, res = _run(hsvd_ctx, ns, ps, Gs, precision=1)
    assert R["status"] == 0, R["statuses"]
    assert max(i["sweeps_fp32"] for i in R["infos"]) >= 1
    for k, (n, p, G) in enumerate(zip(ns, ps, Gs)):
        spread, ref = ordering_spread(G, int(p), block=32)
        e = compare(res[k], ref, int(p))
        gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
        assert e["sigma_norm"] <= 1e-12 and e["U"] <= gate and e["V"] <= gate, (k, n, p, e, spread)
        r = dict(res[k])
        r["sweeps"] = res[k]["sweeps"] + R["infos"][k]["sweeps_fp32"]
        pins.check_invariants(G, int(p), r, tol=1e-15 * n)


def test_batched_mixed_edge_and_no_v(hsvd_ctx):
    """Mixed batch with n = 1, definite signatures and a rank-deficient
    problem (failure local to it), and without V: sigma equal to the run with
    V."""
    g = np.random.Generator(np.random.PCG64(5))
    Gs = [g.standard_normal((n, n)) for n in (1, 7, 64, 65, 130)]
    Gs[3][:, 5] = Gs[3][:, 9]  # duplicate columns: numerically rank deficient
    ns = np.array([1, 7, 64, 65, 130], np.int32)
    ps = np.array([1, 0, 64, 30, 65], np.int32)
    R, res = _run(hsvd_ctx, ns, ps, Gs, precision=1)
    say("mixed edge statuses", R["statuses"], "sweeps", R["sweeps"], [i["sweeps_fp32"] for i in R["infos"]],
        "restarts", [i["fp64_restart"] for i in R["infos"]])
    from paper_1008_1371_amd import hsvd as H
    assert [int(x) for x in R["statuses"]][:3] == [0, 0, 0] and int(R["statuses"][4]) == 0
    assert int(R["statuses"][3]) in (0, H.E_RANK)
    for k in (0, 1, 2, 4):
        ref = oracle.hsvd(Gs[k], int(ps[k]))
        assert np.allclose(np.sort(res[k]["sigma"]), np.sort(ref["sigma"]), rtol=1e-12, atol=0)
    R2, res2 = _run(hsvd_ctx, ns, ps, Gs, precision=1, want_v=0)
    for k in (0, 1, 2, 4):
        assert np.allclose(np.sort(res2[k]["sigma"]), np.sort(res[k]["sigma"]), rtol=1e-12, atol=0)
