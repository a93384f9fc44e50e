"""The FP64 block path and the mixed path at n = 4096 against the oracle's
stored result on the same input (GPU).

The oracle's full-size results (block ordering b = 32, modified modulus, tol
= 1e-15 n) come from tests/golden/make_oracle_n4096.py, which runs only the
oracle: sigma and lambda of every column, U and V on a sample of canonical
columns (8 per J class), and two spreads of the oracle itself on the same
input:
  twin      -- the oracle on G with its rows reversed: the same ordering, only
               the summation order differs;
  ordering  -- the oracle with the round-robin ordering: another trajectory.
Both converge through the stop rule of eq. (4.2) at tol = 1e-15 n, which
leaves the off-diagonal level of the final Gram matrix at up to tol, so two
converged iterates differ in U and V by about that level over the relative
gaps of the spectrum; at n = 4096 that is far above 1e-12, for the oracle's
own twins as for the library.  The singular values move by that level too
where they cluster: the oracle's two orderings differ by 5e-13 normwise at
n = 4096 (tol = 4.1e-12).  The FP64 block path follows the oracle's
trajectory; the mixed path takes its own (FP32 sweeps first) and is held to
the spread between two trajectories, as for U and V.  The gates are:
  sigma normwise, FP64 path      <= 1e-12;
  sigma normwise, mixed path     <= max(1e-12, 10 x the oracle's ordering spread);
  sigma componentwise            <= max(1e-12, 10 x the oracle's largest spread);
  U and V over the sample        <= max(1e-12, 10 x the oracle's largest spread).
"""
import json
import os

import numpy as np
import pytest

from gpu_util import check_invariants_gpu, say
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
WORKLOADS = ["colscaled4096", "graded4096_k1e6_p0.5"]


def _fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_oracle_n4096.py {name})")
    z = np.load(path)
    fx = {k: z[k] for k in z.files if k != "meta"}
    fx["meta"] = json.loads(str(z["meta"]))
    return fx


def _vs_fixture(fx, R, p):
    import torch
    s = R["sigma"].cpu().numpy()
    o1 = np.r_[np.argsort(-s[:p], kind="stable"), p + np.argsort(-s[p:], kind="stable")]
    s0, s1 = fx["sigma"][fx["order"]], s[o1]
    cols = fx["cols"]
    sel = torch.as_tensor(o1[cols], device=R["U"].device)
    U0, V0 = fx["U"], fx["V"]
    U1 = R["U"][:, sel].cpu().numpy()
    V1 = R["V"][:, sel].cpu().numpy()
    rows = np.argmax(np.abs(U0), axis=0)
    k = np.arange(cols.size)
    flip = np.sign(U0[rows, k]) * np.sign(U1[rows, k])
    flip[flip == 0] = 1.0
    U1, V1 = U1 * flip, V1 * flip
    return dict(sigma_norm=float(np.linalg.norm(s1 - s0) / np.linalg.norm(s0)),
                sigma_max=float(np.max(np.abs(s1 - s0) / s0)),
                # root mean square over the sampled columns of the per-column
                # relative differences (the measure of the stored spreads)
                U=float(np.sqrt(np.mean((np.linalg.norm(U1 - U0, axis=0) / np.linalg.norm(U0, axis=0)) ** 2))),
                V=float(np.sqrt(np.mean((np.linalg.norm(V1 - V0, axis=0) / np.linalg.norm(V0, axis=0)) ** 2))),
                lam_norm=float(np.linalg.norm(np.sort(R["lam"].cpu().numpy()) - np.sort(fx["lam"])) /
                               np.linalg.norm(fx["lam"])))


def _oracle_spread(fx):
    m = fx["meta"]
    out = {}
    for key in ("sigma_max", "sigma_norm"):
        out[key] = max(m["twin"][key], m["ordering_spread"][key])
    # the spreads over the same sampled columns as the comparison
    for key, cols in (("U", "U_cols"), ("V", "V_cols")):
        out[key] = max(float(np.linalg.norm(m[s][cols]) / np.sqrt(len(m[s][cols])))
                       for s in ("twin", "ordering_spread"))
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", WORKLOADS)
@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_vs_oracle(hsvd_ctx, name, precision):
    import torch

    from paper_1008_1371_amd import hsvd as H
    fx = _fixture(name)
    G, p = W.workload(name)
    n = G.shape[0]
    assert (n, p) == (fx["meta"]["n"], fx["meta"]["p"])
    Gt = torch.from_numpy(G).cuda()
    R = H.hsvd_solve(hsvd_ctx, Gt, p, H.hsvd_default_params(algo=H.BLOCK, precision=precision), check=False)
    i = R["info"]
    say(name, "precision", precision, "status", R["status"], "sweeps", i["sweeps_fp32"], i["sweeps"],
        "oracle sweeps", fx["meta"]["sweeps"], "reorth", i["reorth_iters"], i["reorth_resid"],
        "restart", i["fp64_restart"], "ms", i["ms_total"])
    assert R["status"] == 0
    e = _vs_fixture(fx, R, p)
    sp = _oracle_spread(fx)
    say("   vs oracle", e)
    say("   oracle spreads (twin / ordering, sampled columns)", sp, "full matrices:",
        {s: {k: fx["meta"][s][k] for k in ("sigma_norm", "sigma_max", "U", "V")}
         for s in ("twin", "ordering_spread")})
    sig_gate = 1e-12 if precision == 0 else max(1e-12, 10 * fx["meta"]["ordering_spread"]["sigma_norm"])
    assert e["sigma_norm"] <= sig_gate, (e, sig_gate)
    assert e["lam_norm"] <= 2 * sig_gate, e
    assert e["sigma_max"] <= max(1e-12, 10 * sp["sigma_max"]), (e, sp)
    gate = max(1e-12, 10 * max(sp["U"], sp["V"]))
    assert e["U"] <= gate and e["V"] <= gate, (e, sp)
    if precision == 1:
        assert i["fp64_restart"] == 0
        assert i["reorth_resid"] <= 16384 * n * 2.0 ** -53
    check_invariants_gpu(Gt, p, R, tol=1e-15 * n, sweeps=i["sweeps"] + i["sweeps_fp32"])


@pytest.mark.timeout(900)
def test_full_size_wide_vs_oracle(hsvd_ctx):
    """The wide block path (b = 64) on colscaled n = 4096 against the oracle's
    stored b = 32 result: another block width is another trajectory, so sigma
    is held to 10x the oracle's ordering spread, like the mixed path."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    name = "colscaled4096"
    fx = _fixture(name)
    G, p = W.workload(name)
    n = G.shape[0]
    Gt = torch.from_numpy(G).cuda()
    R = H.hsvd_solve(hsvd_ctx, Gt, p, H.hsvd_default_params(algo=H.BLOCK, block=64), check=False)
    i = R["info"]
    say(name, "b = 64 status", R["status"], "sweeps", i["sweeps"], "oracle (b = 32) sweeps", fx["meta"]["sweeps"],
        "ms", i["ms_total"])
    assert R["status"] == 0 and i["block"] == 64
    e = _vs_fixture(fx, R, p)
    sp = _oracle_spread(fx)
    say("   vs oracle", e)
    assert e["sigma_norm"] <= max(1e-12, 10 * fx["meta"]["ordering_spread"]["sigma_norm"]), e
    assert e["sigma_max"] <= max(1e-12, 10 * sp["sigma_max"]), (e, sp)
    gate = max(1e-12, 10 * max(sp["U"], sp["V"]))
    assert e["U"] <= gate and e["V"] <= gate, (e, sp)
    check_invariants_gpu(Gt, p, R, tol=1e-15 * n, sweeps=i["sweeps"])
