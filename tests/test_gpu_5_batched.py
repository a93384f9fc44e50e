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


@pytest.mark.parametrize("batch_mode", [0, 1])
def test_batched_mixed_vs_oracle(hsvd_ctx, batch_mode):
    """Mixed precision over a batch: FP32 block sweeps (each problem leaving
    them by its own switch rule), the J-re-orthogonalisation, FP64
    refinement; in one persistent launch (batch_mode 0: each workgroup runs
    the whole mixed solve of its problem) or in grouped launches (1).  Each
    problem against the FP64 oracle: sigma to 1e-12, U and V to 10x the
    ordering spread (the mixed trajectory is its own); the final
    re-orthogonalisation residual within its accepted bound."""
    from parity import ordering_spread
    ns, ps, Gs = W.batch(30, lo=8, hi=200, seed_sizes=78, seed_g=9100)
    say("batched mixed", batch_mode, list(ns))
    R, res = _run(hsvd_ctx, ns, ps, Gs, precision=1, batch_mode=batch_mode)
    assert R["status"] == 0, R["statuses"]
    assert max(i["sweeps_fp32"] for i in R["infos"]) >= 1
    U64 = np.finfo(np.float64).eps / 2
    for k, i in enumerate(R["infos"]):
        if not i["fp64_restart"]:
            assert i["reorth_resid"] <= 16384 * ns[k] * U64, (k, i["reorth_resid"])
    for k, (n, p, G) in enumerate(zip(ns, ps, Gs)):
        spread, ref = ordering_spread(G, int(p), block=32)
        e = compare(res[k], ref, int(p))
        gate = max(1e-12, 10 * max(spread["U"], spread["V"]))
        assert e["sigma_norm"] <= 1e-12 and e["U"] <= gate and e["V"] <= gate, (k, n, p, e, spread)
        r = dict(res[k])
        r["sweeps"] = res[k]["sweeps"] + R["infos"][k]["sweeps_fp32"]
        pins.check_invariants(G, int(p), r, tol=1e-15 * n)


@pytest.mark.parametrize("batch_mode", [0, 1])
def test_batched_mixed_edge_and_no_v(hsvd_ctx, batch_mode):
    """Mixed batch with n = 1, definite signatures and a rank-deficient
    problem (failure local to it), and without V: sigma equal to the run with
    V."""
    g = np.random.Generator(np.random.PCG64(5))
    Gs = [g.standard_normal((n, n)) for n in (1, 7, 64, 65, 130)]
    Gs[3][:, 5] = Gs[3][:, 9]  # duplicate columns: numerically rank deficient
    ns = np.array([1, 7, 64, 65, 130], np.int32)
    ps = np.array([1, 0, 64, 30, 65], np.int32)
    R, res = _run(hsvd_ctx, ns, ps, Gs, precision=1, batch_mode=batch_mode)
    say("mixed edge statuses", R["statuses"], "sweeps", R["sweeps"], [i["sweeps_fp32"] for i in R["infos"]],
        "restarts", [i["fp64_restart"] for i in R["infos"]])
    from paper_1008_1371_amd import hsvd as H
    assert [int(x) for x in R["statuses"]][:3] == [0, 0, 0] and int(R["statuses"][4]) == 0
    assert int(R["statuses"][3]) in (0, H.E_RANK)
    for k in (0, 1, 2, 4):
        ref = oracle.hsvd(Gs[k], int(ps[k]))
        assert np.allclose(np.sort(res[k]["sigma"]), np.sort(ref["sigma"]), rtol=1e-12, atol=0)
    R2, res2 = _run(hsvd_ctx, ns, ps, Gs, precision=1, want_v=0, batch_mode=batch_mode)
    for k in (0, 1, 2, 4):
        assert np.allclose(np.sort(res2[k]["sigma"]), np.sort(res[k]["sigma"]), rtol=1e-12, atol=0)


def _packed(R):
    out = {}
    for k in ("sigma", "lam", "U", "V"):
        out[k] = R[k].cpu().numpy() if R[k] is not None else None
    return out


@pytest.mark.parametrize("ordering,want_v", [("modmod", 1), ("roundrobin", 1), ("modmod", 0)])
def test_batched_persistent_equals_grouped(hsvd_ctx, ordering, want_v):
    """FP64 problems with n <= 256 run in one persistent launch (batch_mode 0)
    or in launches grouped by bordered order (batch_mode 1): the same building
    blocks with the same arithmetic in the same order, so the results are
    bit-identical, statuses and counters included.  Mixed with problems above
    256 (grouped in both modes) and a rank failure."""
    from paper_1008_1371_amd import hsvd as H
    ns, ps, Gs = W.batch(120, seed_sizes=81, seed_g=9300)
    g = np.random.Generator(np.random.PCG64(12))
    for n in (300, 257):
        Gs.append(g.standard_normal((n, n)))
    ns = np.r_[ns, [300, 257]].astype(np.int32)
    ps = np.r_[ps, [100, 257]].astype(np.int32)
    Gs[5] = Gs[5].copy()
    Gs[5][:, 0] = 0.0  # rank failure in one problem only
    o = H.MODMOD if ordering == "modmod" else H.ROUNDROBIN
    outs = []
    for mode in (0, 1):
        R, _ = _run(hsvd_ctx, ns, ps, Gs, ordering=o, want_v=want_v, batch_mode=mode)
        outs.append((R, _packed(R)))
    (R0, P0), (R1, P1) = outs
    say("persistent vs grouped", ordering, "want_v", want_v, "statuses", np.bincount(R0["statuses"] + 3))
    assert np.array_equal(R0["statuses"], R1["statuses"])
    assert R0["statuses"][5] == -3 and (np.delete(R0["statuses"], 5) == 0).all()
    for key in ("sweeps", "rotations", "skips", "steps", "active_pairs", "code", "r", "ldg", "block"):
        a = [i[key] for i in R0["infos"]]
        b = [i[key] for i in R1["infos"]]
        assert a == b, key
    for k in ("sigma", "lam", "U", "V"):
        if P0[k] is None:
            assert P1[k] is None
            continue
        ok = np.isfinite(P1[k])
        assert np.array_equal(P0[k][ok], P1[k][ok]), k


@pytest.mark.timeout(600)
def test_batched_persistent_full_size_matches_grouped(hsvd_ctx):
    """The 10^4-problem workload (n ~ U{8..256}) through both modes: the
    persistent launch reproduces the grouped launches bit for bit."""
    from paper_1008_1371_amd import hsvd as H
    ns, ps, Gs = W.batch(10000)
    P = []
    for mode in (0, 1):
        R, _ = _run(hsvd_ctx, ns, ps, Gs, batch_mode=mode)
        assert R["status"] == 0
        P.append((R, _packed(R)))
        say("mode", mode, "ms", R["infos"][0]["ms_total"], "max sweeps", int(R["sweeps"].max()))
    assert np.array_equal(P[0][0]["sweeps"], P[1][0]["sweeps"])
    for k in ("sigma", "lam", "U", "V"):
        assert np.array_equal(P[0][1][k], P[1][1][k]), k


def test_batched_persistent_widths_bit_identical(tmp_path, monkeypatch):
    """The persistent kernel's workgroup width (256, 512 or 1024 threads per
    problem; the autotuner's choice, fixed here through the tuning cache that
    a new context reads) does not change the results: each width reproduces
    the grouped launches bit for bit.  Then the autotuner picks one of the
    three for this batch's size bucket."""
    from paper_1008_1371_amd import hsvd as H
    ns, ps, Gs = W.batch(64, seed_sizes=83, seed_g=9400)
    ns[0] = 256  # the batch's largest order sets the bucket (192, 256]
    Gs[0] = np.random.Generator(np.random.PCG64(3)).standard_normal((256, 256))
    ref = None
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("HSVD_AUTOTUNE_CACHE", str(cache))
    for threads in (None, 256, 512, 1024):
        if threads is not None:
            cache.write_text('{"entries": [{"batched_bucket": 3, "threads": %d}]}' % threads)
        with H.Context(0) as ctx:
            R, _ = _run(ctx, ns, ps, Gs, batch_mode=0 if threads else 1)
            P = _packed(R)
        assert R["status"] == 0
        if ref is None:
            ref = (R, P)
            continue
        say("width", threads, "bit-identical to grouped")
        assert np.array_equal(R["sweeps"], ref[0]["sweeps"])
        for k in ("sigma", "lam", "U", "V"):
            assert np.array_equal(P[k], ref[1][k]), (threads, k)
    cache.unlink()
    with H.Context(0) as ctx:
        best, ms = H.hsvd_autotune_batched(ctx, ns, ps)
        say("autotune widths (ms)", ms, "best", best)
        assert best in (256, 512, 1024) and all(v > 0 for v in ms.values())
        assert best == min(ms, key=ms.get)
        assert '"threads": %d' % best in cache.read_text()
        # the sweep schedule per precision, which batch_mode 2 (the default)
        # then takes: the same results as asking for that schedule
        for prec in (H.FP64, H.MIXED):
            sched = H.hsvd_batched_schedule(ctx, prec)
            say("autotuned schedule", prec, ("persistent", "grouped")[sched])
            assert sched in (0, 1)
            assert '"batched_schedule": %d, "mode": %d' % (prec, sched) in cache.read_text()
            Ra, _ = _run(ctx, ns, ps, Gs, precision=prec)
            Rb, _ = _run(ctx, ns, ps, Gs, precision=prec, batch_mode=sched)
            Pa, Pb = _packed(Ra), _packed(Rb)
            for k in ("sigma", "lam", "U", "V"):
                assert np.array_equal(Pa[k], Pb[k]), (prec, k)


def test_batched_persistent_mixed_widths_bit_identical(tmp_path, monkeypatch):
    """Mixed precision in the persistent launch: the workgroup width does not
    change the results (every phase, the re-orthogonalisation products
    included, has width-independent arithmetic), and the FP64 restart of a
    problem whose FP32 phase meets a rank flag stays local to it."""
    from paper_1008_1371_amd import hsvd as H
    ns, ps, Gs = W.batch(48, seed_sizes=85, seed_g=9500)
    ns[0] = 256
    Gs[0] = np.random.Generator(np.random.PCG64(4)).standard_normal((256, 256))
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("HSVD_AUTOTUNE_CACHE", str(cache))
    ref = None
    for threads in (256, 512, 1024):
        cache.write_text('{"entries": [{"batched_bucket": 3, "threads": %d}]}' % threads)
        with H.Context(0) as ctx:
            R, _ = _run(ctx, ns, ps, Gs, precision=1, batch_mode=0)
            P = _packed(R)
        say("mixed persistent width", threads, "status", R["status"], "fp32 sweeps",
            max(i["sweeps_fp32"] for i in R["infos"]), "restarts", sum(i["fp64_restart"] for i in R["infos"]))
        assert R["status"] == 0
        if ref is None:
            ref = (R, P)
            continue
        assert np.array_equal(R["sweeps"], ref[0]["sweeps"])
        for key in ("sweeps_fp32", "reorth_iters", "fp64_restart", "reorth_resid", "rotations"):
            assert [i[key] for i in R["infos"]] == [i[key] for i in ref[0]["infos"]], (threads, key)
        for k in ("sigma", "lam", "U", "V"):
            assert np.array_equal(P[k], ref[1][k]), (threads, k)
