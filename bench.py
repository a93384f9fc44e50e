#!/usr/bin/env python3
"""Benchmark: time-to-solution and solves/s of the one-sided Jacobi HSVD on one MI355X.

One "step" is one complete solve (all sweeps until the stop rule of eq. 4.2,
with Sigma, U, V and lambda extracted) of the named workload, with the input
already resident in HBM.  The headline compares the mixed-precision path
(FP32 MFMA block sweeps, FP64 J-re-orthogonalisation, FP64 refinement) with the
FP64 block path on the same input; `value` is the mixed path's throughput and
the FP64 path's is reported beside it.  The JSON line also carries the roofline
of the dominant kernel (HIP events around every launch on the library's
stream during the timed solves), accuracy invariants of the last solve, the
CPU oracle timed on a bounded sample of the same workload, and optionally the
batched solver's throughput on 10,000 small problems.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "HSVD time-to-solution n=4096 (mixed vs FP64 GPU) at rel err ≤1e-12; solves/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and, in a
# second run, WRITE_SIZE (KiB per dispatch, averaged over all launches of each
# kernel class in one mixed colscaled4096 solve), each scaled by what the same
# counter reads for a plain 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0).  The averages hold only for the sources they were taken on (the
# kernels, and the host code that sets their launch shapes and the solve's
# trajectory): when the SHA-256 over these files changes the roofline reports
# traffic as null.
MEASURED_TRAFFIC = {
    "workload": "colscaled4096",
    "mode": "mixed",
    "sources": ["paper_1008_1371_amd/csrc/block_kernels.hip", "paper_1008_1371_amd/csrc/block_device.h",
                "paper_1008_1371_amd/csrc/api.hip", "paper_1008_1371_amd/csrc/internal.h"],
    "sha256": "54ce685e23de08f1ffb633d6140eefc89c1d8bfb733bdb02c46b1f8449305e53",
    "bytes_per_launch": {
        "block_gram_kernel<float>": (32853.2 * 2.0 + 5120.0 * 1.0) * 1024,
        "block_inner_kernel<float>": (22295.7 * 2.0 + 37575.6 * 1.0) * 1024,
        "block_update_kernel<float>": (20340.1 * 2.0 + 35950.4 * 1.0) * 1024,
        "block_gram_kernel<double>": (65593.5 * 2.0 + 10240.0 * 1.0) * 1024,
        "block_inner_kernel<double>": (27488.0 * 2.0 + 37493.5 * 1.0) * 1024,
        "block_update_kernel<double>": (20033.4 * 2.0 + 35511.7 * 1.0) * 1024,
    },
}


def measured_traffic(kernel, workload, mode):
    """Counter-based HBM bytes per launch of `kernel`, or None when the
    measurement does not apply (other workload or solve mode, other kernel,
    changed source)."""
    import hashlib
    t = MEASURED_TRAFFIC
    if workload != t["workload"] or mode != t["mode"] or kernel not in t["bytes_per_launch"]:
        return None
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    try:
        for src in t["sources"]:
            with open(os.path.join(root, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    if h.hexdigest() != t["sha256"]:
        return None
    return t["bytes_per_launch"][kernel]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="colscaled4096")
    ap.add_argument("--mode", default="both", choices=["both", "fp64", "mixed", "pairwise", "batched"],
                    help="both: mixed is the headline, FP64 block timed beside it; batched: only the batched "
                         "solver's persistent launch (FP64 and mixed, untuned width; profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the bounded oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--batched", type=int, default=10000,
                    help="also time the batched solver on this many small problems (0: skip)")
    ap.add_argument("--block", type=int, default=0, choices=[0, 32, 64],
                    help="block width of the FP64 block path (0: the library's default, 32); 64 runs the wide "
                         "block path, FP64 only")
    ap.add_argument("--persistent", type=int, default=0, choices=[0, 1, 2],
                    help="pairwise path: 0 one launch per step (graph replay), 1 one persistent launch with "
                         "per-column readiness between steps, 2 the same with a grid barrier per step")
    ap.add_argument("--also", default="graded4096_k1e6_p0.5",
                    help="a second workload timed beside the headline (mixed and FP64, errors against its stored "
                         "oracle result); empty: none")
    ap.add_argument("--inner-sweeps", type=int, default=0,
                    help="block modes: 0 = block-oriented method; k > 0 = full-block method with at most "
                         "k inner sweeps per pivot block")
    ap.add_argument("--no-v", action="store_true",
                    help="eigenvalues / singular values and U only: V is not returned (the mixed path "
                         "still carries V internally through its FP32 phase)")
    ap.add_argument("--max-sweeps", type=int, default=0,
                    help="stop each solve after this many sweeps (profiling runs only)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB 8 times (scale for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def accuracy(G, p, R, lam=None):
    """Invariants of a solve, in FP64 on the GPU (torch matmuls).  With the
    prescribed spectrum lam of an eigen workload, also the relative errors of
    the computed eigenvalues sigma^2 j and d(U) = ||I - U^T U||_F (Sec. 5)."""
    import numpy as np
    import torch
    n = G.shape[0]
    U, V, s = R["U"], R["V"], R["sigma"]
    j = torch.ones(n, dtype=torch.float64, device=G.device)
    j[p:] = -1.0
    UtU = U.t() @ U
    # the stop rule bounds the cosines the solver computes by tol; recomputed
    # from the returned U they may exceed it by rounding (the tests allow 2 tol)
    out = {"max_offdiag_UtU": (UtU - torch.diag(torch.diagonal(UtU))).abs().max().item(),
           "tol": 1e-15 * n, "bound": 2e-15 * n}
    if lam is not None:
        got = np.sort((s * s * j).cpu().numpy())
        want = np.sort(lam)
        rel = np.abs(got - want) / np.abs(want)
        out["eig_rel_max"] = float(rel.max())
        out["eig_rel_mean"] = float(rel.mean())
        out["eig_rel_bound"] = 20 * n * float(np.finfo(np.float64).eps / 2)
        out["dU"] = torch.linalg.matrix_norm(torch.eye(n, dtype=torch.float64, device=G.device) - UtU).item()
    if V is not None:
        VtJV = V.t() @ (V * j[:, None])
        vn = torch.linalg.matrix_norm(V, ord=2).item() ** 2
        out["VtJV_resid"] = (torch.linalg.matrix_norm(VtJV - torch.diag(j)) / vn).item()
        out["GV_US_resid"] = (torch.linalg.matrix_norm(G @ V - U * s[None, :]) /
                              (torch.linalg.matrix_norm(G) * max(1.0, vn ** 0.5))).item()
    return out


def canonical_diff(ref, got, p):
    """Relative differences of `got` from `ref` (sigma, U, V; several results
    are correct): within each J class (physical columns [0, p) and [p, n))
    the columns are ordered by sigma descending, then each column pair of
    `got` is sign-aligned to `ref` at the row where ref's u is largest."""
    import torch

    def order(s):
        idx = torch.arange(s.numel(), device=s.device)
        return torch.cat([idx[:p][torch.argsort(-s[:p], stable=True)],
                          idx[p:][torch.argsort(-s[p:], stable=True)]])
    o0, o1 = order(ref["sigma"]), order(got["sigma"])
    s0, s1 = ref["sigma"][o0], got["sigma"][o1]
    U0, U1 = ref["U"][:, o0], got["U"][:, o1]
    cols = torch.arange(U0.shape[1], device=U0.device)
    rows = U0.abs().argmax(dim=0)
    flip = torch.sign(U0[rows, cols]) * torch.sign(U1[rows, cols])
    flip[flip == 0] = 1.0
    out = {"sigma_norm": (torch.linalg.vector_norm(s1 - s0) / torch.linalg.vector_norm(s0)).item(),
           "sigma_max": ((s1 - s0).abs() / s0).max().item(),
           "U": (torch.linalg.matrix_norm(U1 * flip - U0) / torch.linalg.matrix_norm(U0)).item()}
    if ref.get("V") is not None and got.get("V") is not None:
        V0, V1 = ref["V"][:, o0], got["V"][:, o1]
        out["V"] = (torch.linalg.matrix_norm(V1 * flip - V0) / torch.linalg.matrix_norm(V0)).item()
    return out


ROOT = os.path.dirname(os.path.abspath(__file__))


def oracle_fixture(workload):
    """The stored oracle result of a full-size workload (written by
    tests/golden/make_oracle_n4096.py, which runs only the oracle), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    fx = {k: z[k] for k in z.files if k != "meta"}
    fx["meta"] = json.loads(str(z["meta"]))
    return fx


def vs_oracle(fx, R, p):
    """The GPU result against the stored oracle result, canonicalised as in
    the tests (each J class by sigma descending; column pairs sign-aligned on
    u at the oracle's largest entry): sigma normwise and componentwise over
    all columns, U and V on the stored sample of columns (per column and over
    the sample)."""
    import numpy as np
    s = R["sigma"].cpu().numpy()
    n = s.size
    o1 = np.r_[np.argsort(-s[:p], kind="stable"), p + np.argsort(-s[p:], kind="stable")]
    s0 = fx["sigma"][fx["order"]]
    s1 = s[o1]
    import torch
    cols = fx["cols"]
    sel = torch.as_tensor(o1[cols], device=R["U"].device)
    U1 = R["U"][:, sel].cpu().numpy()
    U0 = fx["U"]
    rows = np.argmax(np.abs(U0), axis=0)
    flip = np.sign(U0[rows, np.arange(cols.size)]) * np.sign(U1[rows, np.arange(cols.size)])
    flip[flip == 0] = 1.0
    U1 = U1 * flip
    out = {"sigma_norm": float(np.linalg.norm(s1 - s0) / np.linalg.norm(s0)),
           "sigma_max": float(np.max(np.abs(s1 - s0) / s0)),
           "U_sample": float(np.linalg.norm(U1 - U0) / np.linalg.norm(U0)),
           "U_col_max": float(np.max(np.linalg.norm(U1 - U0, axis=0)))}
    if R.get("V") is not None:
        V1 = R["V"][:, sel].cpu().numpy() * flip
        V0 = fx["V"]
        out["V_sample"] = float(np.linalg.norm(V1 - V0) / np.linalg.norm(V0))
        out["V_col_max"] = float(np.max(np.linalg.norm(V1 - V0, axis=0) / np.linalg.norm(V0, axis=0)))
    out["sampled_columns"] = int(cols.size)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(G_np, p, block, target_s, fx, workload):
    """The oracle (the FP64 path's ordering: block b, modified modulus) timed
    on the host cores, on two bounded samples of the same workload:
      A: the first outer steps of the solve on the workload's input, where
         nearly every pair visit rotates;
      B: the first outer steps on an input of the same shape and column
         scaling whose columns are orthogonal, where every pair visit is
         skipped (dot product and test only).
    Their times give the oracle's cost per rotated and per skipped pair visit
    (two equations, two unknowns), and the full solve is priced with the
    oracle's own counts of rotated and skipped visits over the whole solve
    (stored with the oracle's full-size result).  Without that result, the
    sample A rate is extrapolated over the steps (an upper bound)."""
    import numpy as np

    import oracle
    from paper_1008_1371_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = G_np.shape[0]
    steps_total = None if fx is None else fx["meta"]["steps"]
    # size the samples from the cost of two steps
    t0 = time.perf_counter()
    oracle.hsvd(G_np, p, max_steps=2, nthreads=threads, block=block)
    per_step = max((time.perf_counter() - t0) / 2, 1e-6)
    sa = int(max(4, target_s * 0.65 / per_step))
    t0 = time.perf_counter()
    A = oracle.hsvd(G_np, p, max_steps=sa, nthreads=threads, block=block)
    tA = time.perf_counter() - t0
    res = {"unit": "solves/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "nproc": os.cpu_count()}
    if fx is None:
        est = tA / max(1, A["steps"]) * (A["steps"] if steps_total is None else steps_total)
        res.update(value=1.0 / est, sample=(f"oracle (block ordering b={block}, FP64) on the first {A['steps']} "
                                            f"outer steps ({tA:.1f} s); no full-size oracle counts stored for "
                                            f"{workload}: rate of those steps only"))
        return res
    # B: orthogonal columns with the workload's column scaling (every visit skipped)
    Q = W.haar(n, seed=W.SEED_Q1)
    Gb = np.asfortranarray(Q * np.sqrt(np.sum(G_np * G_np, axis=0))[None, :])
    sb = int(max(4, sa))
    t0 = time.perf_counter()
    B = oracle.hsvd(Gb, p, max_steps=sb, nthreads=threads, block=block)
    tB = time.perf_counter() - t0
    c_skip = tB / max(1, B["skips"] + B["rotations"])
    c_rot = max(tA - A["skips"] * c_skip, 0.0) / max(1, A["rotations"])
    R_tot, S_tot = fx["meta"]["rotations"], fx["meta"]["skips"]
    est = R_tot * c_rot + S_tot * c_skip
    res.update(value=1.0 / est,
               sample=(f"oracle (block ordering b={block}, FP64, {threads} threads): sample A = first {A['steps']} "
                       f"outer steps on {workload} ({A['rotations']} rotated / {A['skips']} skipped pair visits, "
                       f"{tA:.1f} s); sample B = first {B['steps']} outer steps on orthogonal columns of the same "
                       f"scaling ({B['skips']} skipped visits, {tB:.1f} s); full solve priced with the oracle's own "
                       f"{R_tot} rotated and {S_tot} skipped visits ({fx['meta']['sweeps']} sweeps): {est:.0f} s"),
               seconds_per_solve=est, rot_visit_us=c_rot * 1e6, skip_visit_us=c_skip * 1e6)
    return res


def roofline(infos, names, peaks, workload, mode):
    """Roofline of the kernel class with the most measured time."""
    nk = len(names)
    ms = [sum(i["kernel_ms"][q] for i in infos) for q in range(nk)]
    q = max(range(nk), key=lambda k: ms[k])
    launches = sum(i["kernel_launches"][q] for i in infos)
    byts = sum(i["kernel_bytes"][q] for i in infos)
    flops = sum(i["kernel_flops"][q] for i in infos)
    avg_s = ms[q] * 1e-3 / launches
    bpl, fpl = byts / launches, flops / launches
    peak_tf = peaks[q]
    if flops > 0 and flops / byts * HBM_PEAK_GBS * 1e9 > peak_tf * 1e12:
        ach = fpl / avg_s / 1e12
        r = {"bound": "mfma", "achieved": ach, "peak": peak_tf, "unit": "TFLOP/s", "frac": ach / peak_tf}
    else:
        ach = bpl / avg_s / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": ach / HBM_PEAK_GBS}
    r.update({"traffic": measured_traffic(names[q], workload, mode), "kernel": names[q], "avg_launch_us": avg_s * 1e6,
              "launches_timed": sum(i["kernel_timed"][q] for i in infos), "launches": launches,
              "bytes_per_launch": bpl, "flops_per_launch": fpl,
              "share_of_solve": ms[q] / sum(i["ms_total"] for i in infos)})
    other = {}
    for k in range(nk):
        L = sum(i["kernel_launches"][k] for i in infos)
        if L:
            kb = sum(i["kernel_bytes"][k] for i in infos)
            kf = sum(i["kernel_flops"][k] for i in infos)
            other[names[k]] = {"avg_launch_us": ms[k] * 1e3 / L, "launches_per_solve": L / len(infos),
                               "ms_per_solve": ms[k] / len(infos),
                               "GB/s": kb / (ms[k] * 1e-3) / 1e9 if ms[k] else None,
                               "TFLOP/s": kf / (ms[k] * 1e-3) / 1e12 if ms[k] and kf else None}
    r["kernels"] = other
    return r


def timed(H, ctx, G, p, prm, out, steps, warmup, check):
    import torch
    for _ in range(warmup):
        H.hsvd_solve(ctx, G, p, prm, out=out, check=check)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        R = H.hsvd_solve(ctx, G, p, prm, out=out, check=check)
        infos.append(R["info"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return 1000.0 * wall / steps, infos, R


def batched_line(H, W, ctx, count, persistent_only=False):
    """The batched solver on `count` Gaussian problems, n ~ U{8..256}, FP64
    and mixed precision, with the sweep schedule and the persistent kernel's
    width the autotuner picks (tuned first, outside the timed runs), and each
    schedule on its own for comparison: one persistent launch, and launches
    grouped by bordered order.  persistent_only: the persistent launch alone,
    FP64 and mixed, at the untuned width (one warm-up and one timed call each).
    """
    import numpy as np
    import torch
    ns, ps, Gs = W.batch(count)
    flat, offs = W.pack_batch(Gs)
    voffs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    Gd = torch.from_numpy(flat).cuda()
    out = {"problems": count, "n_range": [int(ns.min()), int(ns.max())]}
    configs = (("fp64_persistent", H.FP64, 0), ("mixed_persistent", H.MIXED, 0))
    if not persistent_only:
        # the persistent kernel's width for this size mix (outside the timed runs)
        best, widths = H.hsvd_autotune_batched(ctx, ns, ps)
        out["persistent_width"] = {"threads": best, "autotune_ms": widths}
        out["schedule"] = {name: ("persistent", "grouped")[H.hsvd_batched_schedule(ctx, prec)]
                           for name, prec in (("fp64", H.FP64), ("mixed", H.MIXED))}
        configs = ((("fp64", H.FP64, 2), ("mixed", H.MIXED, 2)) + configs[:1] + (("fp64_grouped", H.FP64, 1),) +
                   configs[1:] + (("mixed_grouped", H.MIXED, 1),))
    for name, prec, mode in configs:
        prm = H.hsvd_default_params(precision=prec, batch_mode=mode)
        H.hsvd_solve_batched(ctx, ns, ps, Gd, offs, voffs, prm)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R = H.hsvd_solve_batched(ctx, ns, ps, Gd, offs, voffs, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # algorithmic flops of a batch, counted as 9 n^3 per sweep and problem
        # (FP32 and FP64 sweeps alike), against the FP64 peak
        sw = np.array([i["sweeps"] + i["sweeps_fp32"] for i in R["infos"]], dtype=np.float64)
        gflop = float((sw * 9.0 * ns.astype(np.float64) ** 3).sum()) / 1e9
        out[name] = {"seconds": dt, "solves_per_s": count / dt, "gflop_algorithmic": gflop,
                     "tflops": gflop / dt / 1e3, "frac_fp64_peak": gflop / dt / 1e3 / FP64_PEAK_TFLOPS,
                     "max_sweeps_fp32": max(i["sweeps_fp32"] for i in R["infos"]),
                     "max_sweeps": int(R["sweeps"].max()), "all_converged": bool((R["statuses"] == 0).all()),
                     "fp64_restarts": sum(i["fp64_restart"] for i in R["infos"])}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1008_1371_amd import hsvd as H
    from paper_1008_1371_amd import workloads as W

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 8}), flush=True)
        return

    H.lib()  # fails loudly if the HIP library is missing
    if args.mode == "batched":
        print(json.dumps({"batched": batched_line(H, W, H.Context(0), args.batched or 10000, True)}), flush=True)
        return
    G_np, p = W.workload(args.workload)
    n = G_np.shape[0]
    # the prescribed spectrum of an eigen workload (cached by the generator)
    lam = None
    if args.workload.startswith("eigen"):
        body = args.workload[5:]
        lam = W.eigen(n, npos=int(body.split("_p")[1]) if "_p" in body else None)[2]
    dev = torch.device("cuda:0")
    G = torch.from_numpy(np.asfortranarray(G_np)).to(dev)
    ctx = H.Context(0)
    out = dict(
        sigma=torch.empty(n, dtype=torch.float64, device=dev),
        U=torch.empty((n, n), dtype=torch.float64, device=dev).t(),
        V=None if args.no_v else torch.empty((n, n), dtype=torch.float64, device=dev).t(),
        **{"lambda": torch.empty(n, dtype=torch.float64, device=dev)},
        perm=torch.empty(n, dtype=torch.int32, device=dev),
    )
    check = args.max_sweeps <= 0
    peaks = [FP64_PEAK_TFLOPS] * 4 + [FP32_PEAK_TFLOPS] * 3 + [FP64_PEAK_TFLOPS]

    def variant(mode):
        # the counter measurements hold for the default variant of a mode only
        return (mode + ("/full-block" if args.inner_sweeps > 0 else "") + ("/no-v" if args.no_v else "") +
                ("/b64" if args.block == 64 else "") +
                (f"/persistent{args.persistent}" if mode == "pairwise" and args.persistent else ""))

    def params(mode):
        prm = H.hsvd_default_params(algo=H.PAIRWISE if mode == "pairwise" else H.BLOCK,
                                    precision=H.MIXED if mode == "mixed" else H.FP64,
                                    want_v=0 if args.no_v else 1,
                                    inner_sweeps=0 if mode == "pairwise" else args.inner_sweeps,
                                    block=args.block if mode == "fp64" else 0,
                                    persistent=args.persistent if mode == "pairwise" else 0)
        if args.max_sweeps > 0:
            prm.max_sweeps = args.max_sweeps
        return prm

    runs = {}
    modes = ["fp64", "mixed"] if args.mode == "both" else [args.mode]
    names = list(H.KERNEL_NAMES)
    if args.block == 64:
        # b = 64 is an FP64 path; its kernel classes are the block-pair GEMMs
        # and the wide inner kernel
        modes = ["fp64"]
        names[1:4] = ["gemm_f64_kernel (block-pair Gram, b = 64)", "wide_inner_kernel",
                      "gemm_f64_kernel (block-pair update, b = 64)"]
    if args.mode == "pairwise" and args.persistent:
        names[0] = "pair_persist_kernel (all sweeps, one launch)"
    results = {}
    for mode in modes:
        ms, infos, R = timed(H, ctx, G, p, params(mode), out, args.steps, args.warmup, check)
        acc = None if args.no_accuracy else accuracy(G, p, R, lam)
        runs[mode] = (ms, infos, acc)
        if not args.no_accuracy:
            # the output buffers are shared between the modes
            results[mode] = {k: (R[k].clone() if R[k] is not None else None) for k in ("sigma", "U", "V")}
    head = "mixed" if "mixed" in runs else modes[0]
    ms, infos, acc = runs[head]
    last = infos[-1]
    line = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "path": f"{head}",
                   "block": last["block"], "ordering": "modmod", "sort": 1, "want_v": 0 if args.no_v else 1,
                   "method": ("pairwise" if head == "pairwise" else
                              "full-block" if args.inner_sweeps > 0 else "block-oriented"),
                   "inner_sweeps": args.inner_sweeps,
                   "tol": 1e-15 * n, "sweeps_fp32": last["sweeps_fp32"], "sweeps_fp64": last["sweeps"],
                   "reorth_iters": last["reorth_iters"], "rotations": last["rotations"],
                   "steps_per_solve": last["steps"]},
        "roofline": roofline(infos, names, peaks, args.workload, variant(head)),
    }
    if acc is not None:
        line["accuracy"] = acc
    for mode, (m_ms, m_infos, m_acc) in runs.items():
        if mode == head:
            continue
        line[mode] = {"value": 1000.0 / m_ms, "ms_per_step": m_ms, "sweeps": m_infos[-1]["sweeps"],
                      "roofline": roofline(m_infos, names, peaks, args.workload, variant(mode)),
                      "accuracy": m_acc}
        line["speedup_vs_" + mode] = m_ms / ms
    if "fp64" in results and "mixed" in results:
        # the mixed path against the FP64 path on the same input
        line["mixed_vs_fp64"] = canonical_diff(results["fp64"], results["mixed"], p)
    fx = oracle_fixture(args.workload) if args.inner_sweeps == 0 else None
    if fx is not None and not args.no_accuracy:
        # both paths against the oracle's stored full-size result, beside the
        # oracle's own spreads on the same input: the twin (same trajectory,
        # rows reversed) and the ordering spread (round-robin vs modified
        # modulus: two converged iterates the stop rule accepts)
        for mode in ("fp64", "mixed"):
            if mode in results:
                line[mode + "_vs_oracle"] = vs_oracle(fx, results[mode], p)
        m = fx["meta"]
        line["oracle_spread"] = {k: {q: m[k][q] for q in ("sigma_norm", "sigma_max", "U", "V")} |
                                 {"U_col_max": max(m[k]["U_cols"]), "V_col_max": max(m[k]["V_cols"])}
                                 for k in ("twin", "ordering_spread")}
    if args.also and args.also != args.workload and args.inner_sweeps == 0 and args.block != 64 \
            and args.mode in ("both", "mixed", "fp64") and not args.no_v and args.max_sweeps <= 0:
        # the second workload: the graded-spectrum matrix of the paper's
        # experiments at n = 4096 (kappa 1e6, p = n/2), both paths, each
        # against the oracle's stored result of the same input
        G2_np, p2 = W.workload(args.also)
        n2 = G2_np.shape[0]
        G2 = torch.from_numpy(np.asfortranarray(G2_np)).to(dev)
        out2 = dict(sigma=torch.empty(n2, dtype=torch.float64, device=dev),
                    U=torch.empty((n2, n2), dtype=torch.float64, device=dev).t(),
                    V=torch.empty((n2, n2), dtype=torch.float64, device=dev).t(),
                    **{"lambda": torch.empty(n2, dtype=torch.float64, device=dev)},
                    perm=torch.empty(n2, dtype=torch.int32, device=dev))
        fx2 = oracle_fixture(args.also)
        also = {"n": n2, "p": p2}
        for mode in ("mixed", "fp64"):
            m_ms, m_infos, R2 = timed(H, ctx, G2, p2, params(mode), out2, args.steps, args.warmup, True)
            also[mode] = {"ms_per_step": m_ms, "solves_per_s": 1000.0 / m_ms, "sweeps": m_infos[-1]["sweeps"],
                          "sweeps_fp32": m_infos[-1]["sweeps_fp32"]}
            if fx2 is not None and not args.no_accuracy:
                also[mode]["vs_oracle"] = vs_oracle(fx2, R2, p2)
        if fx2 is not None:
            m2 = fx2["meta"]
            also["oracle_spread"] = {k: {q: m2[k][q] for q in ("sigma_norm", "sigma_max", "U", "V")}
                                     for k in ("twin", "ordering_spread") if k in m2}
        line["also"] = {args.also: also}
    if args.batched > 0:
        line["batched"] = batched_line(H, W, ctx, args.batched)
    if not args.no_cpu_baseline:
        block = (runs["fp64"][1] if "fp64" in runs else infos)[-1]["block"]
        line["cpu_baseline"] = cpu_baseline(G_np, p, block, args.cpu_seconds, fx, args.workload)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
