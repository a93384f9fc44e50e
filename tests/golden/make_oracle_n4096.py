"""Writes the oracle fixtures of the full-size parity tests (n = 4096).

Calls only ``oracle/`` (and the seeded input generators): for each workload
the oracle's block-ordered FP64 solve (b = 32, modified modulus, tol =
1e-15 n, the configuration of the block path it checks) is run three times:

* the reference run, whose sigma, lambda and a sample of canonicalised U and
  V columns are stored;
* its twin, the same run on G with the rows reversed (U's rows un-reversed
  afterwards): the same trajectory with another summation order, so the
  difference is the rounding spread of one trajectory;
* the round-robin run: another trajectory to convergence, so the difference
  is the spread between two converged iterates that the stop rule of
  eq. (4.2) accepts at this tolerance.

Both spreads are stored for the whole matrices and for the sampled columns.
The oracle's counters (sweeps, rotations, skips) and its wall time are
stored too.

Usage: python tests/golden/make_oracle_n4096.py <workload> [threads]
       workloads: colscaled4096, graded4096_k1e6_p0.5
Takes about 15-25 minutes per oracle run on 8 host cores.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1008_1371_amd import workloads as W  # noqa: E402

PER_CLASS = 8  # sampled columns per J class


def canon_order(sigma, p):
    """Canonical column order: within each J class by sigma descending."""
    n = sigma.size
    pos = sorted(range(p), key=lambda c: -sigma[c])
    neg = sorted(range(p, n), key=lambda c: -sigma[c])
    return np.array(pos + neg, dtype=np.int64)


def sample_columns(n, p):
    """Positions (in canonical order) of the sampled columns: PER_CLASS evenly
    spaced in each J class, first and last included."""
    out = []
    for lo, hi in ((0, p), (p, n)):
        if hi > lo:
            k = min(PER_CLASS, hi - lo)
            out.extend(np.unique(np.round(np.linspace(lo, hi - 1, k)).astype(np.int64)).tolist())
    return np.array(out, dtype=np.int64)


def spread(a, b, p, cols):
    """Differences of run b against run a (canonicalised, sign-aligned on U)."""
    oa, ob = canon_order(a["sigma"], p), canon_order(b["sigma"], p)
    sa, sb = a["sigma"][oa], b["sigma"][ob]
    Ua, Ub = a["U"][:, oa], b["U"][:, ob]
    Va, Vb = a["V"][:, oa], b["V"][:, ob]
    n = sa.size
    rows = np.argmax(np.abs(Ua), axis=0)
    flip = np.sign(Ua[rows, np.arange(n)]) * np.sign(Ub[rows, np.arange(n)])
    flip[flip == 0] = 1.0
    Ub = Ub * flip
    Vb = Vb * flip
    du = np.linalg.norm(Ub - Ua, axis=0)
    dv = np.linalg.norm(Vb - Va, axis=0) / np.linalg.norm(Va, axis=0)
    return dict(
        sigma_norm=float(np.linalg.norm(sb - sa) / np.linalg.norm(sa)),
        sigma_max=float(np.max(np.abs(sb - sa) / sa)),
        U=float(np.linalg.norm(Ub - Ua) / np.linalg.norm(Ua)),
        V=float(np.linalg.norm(Vb - Va) / np.linalg.norm(Va)),
        U_cols=du[cols].tolist(),
        V_cols=dv[cols].tolist(),
    )


def run(G, p, threads, **kw):
    t0 = time.time()
    R = oracle.hsvd(G, p, block=32, nthreads=threads, **kw)
    R["seconds"] = time.time() - t0
    assert R["status"] == oracle.OK, R["status"]
    print(f"  oracle {kw or 'modmod'}: {R['seconds']:.1f} s, {R['sweeps']} sweeps", flush=True)
    return R


def main(name, threads):
    G, p = W.workload(name)
    n = G.shape[0]
    print(name, n, p, flush=True)
    ref = run(G, p, threads)
    twin = run(np.asfortranarray(G[::-1, :]), p, threads)
    twin["U"] = twin["U"][::-1, :]
    rr = run(G, p, threads, ordering="roundrobin")
    o = canon_order(ref["sigma"], p)
    cols = sample_columns(n, p)
    Us = ref["U"][:, o[cols]]
    Vs = ref["V"][:, o[cols]]
    meta = dict(workload=name, n=n, p=p, tol=ref["tol"], block=32, ordering="modmod",
                sweeps=ref["sweeps"], rotations=int(ref["rotations"]), skips=int(ref["skips"]),
                steps=int(ref["steps"]), seconds=ref["seconds"], threads=threads,
                twin=spread(ref, twin, p, cols), ordering_spread=spread(ref, rr, p, cols),
                rr_sweeps=rr["sweeps"], per_class=PER_CLASS)
    out = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(out, sigma=ref["sigma"], lam=ref["lam"], perm=ref["perm"], order=o,
                        cols=cols, U=Us, V=Vs, meta=np.array(json.dumps(meta)))
    print(json.dumps({k: v for k, v in meta.items()}, indent=1), flush=True)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
