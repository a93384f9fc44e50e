"""Block path with column blocks of b = 64 (the wide block path, FP64) against
the oracle's block ordering with b = 64 (GPU)."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import run_lib, say
from parity import compare, twin_spread
from paper_1008_1371_amd import workloads as W
from test_gpu_3_block import _oracle_block_trace

pytestmark = pytest.mark.gpu
B = 64


@pytest.mark.parametrize("r", [128, 256, 1024])
@pytest.mark.parametrize("ordering", ["modmod", "roundrobin"])
def test_wide_block_trace_bit_exact(hsvd_ctx, r, ordering):
    import torch

    from paper_1008_1371_amd import hsvd as H
    nb = r // B
    steps = 2 * nb + 1
    want = _oracle_block_trace(ordering, r, B, steps)
    say("block_trace b=64", ordering, r, steps, want.shape)
    buf = torch.empty(want.size, dtype=torch.int32, device="cuda:0")
    st = H.lib().hsvd_block_trace(hsvd_ctx.handle, H.MODMOD if ordering == "modmod" else H.ROUNDROBIN, r, B,
                                  steps, H._ptr(buf))
    assert st == 0
    assert np.array_equal(buf.cpu().numpy().reshape(-1, 2), want)


def _gate(G, p, res, ref, uv_gate=1e-12):
    assert res["status"] == 0, res["status"]
    assert res["info"]["block"] == B
    e = compare(res, ref, p)
    say("   errors", e, "sweeps lib/orc", res["info"]["sweeps"], ref["sweeps"])
    assert e["sigma_norm"] <= 1e-12, e
    assert e["U"] <= uv_gate and e.get("V", 0.0) <= uv_gate, e
    pins.check_invariants(G, p, res, tol=ref["tol"])


@pytest.mark.parametrize("n,p", [(1, 1), (5, 0), (100, 37), (128, 64), (128, 128), (200, 77), (333, 300),
                                 (512, 256)])
@pytest.mark.parametrize("ordering", ["modmod", "roundrobin"])
def test_wide_small(hsvd_ctx, n, p, ordering):
    G = W.colscaled(n, 2.0, seed=160 + n)
    say("wide block", n, p, ordering)
    ref = oracle.hsvd(G, p, block=B, ordering=ordering)
    res = run_lib(hsvd_ctx, G, p, algo=2, block=B, ordering=0 if ordering == "modmod" else 1)
    _gate(G, p, res, ref)


def test_wide_unsorted_no_v_and_errors(hsvd_ctx):
    from paper_1008_1371_amd import hsvd as H
    G, p = W.workload("gauss128")
    ref = oracle.hsvd(G, p, block=B, sort=False)
    res = run_lib(hsvd_ctx, G, p, algo=2, block=B, sort=0)
    _gate(G, p, res, ref)
    res2 = run_lib(hsvd_ctx, G, p, algo=2, block=B, want_v=0)
    e = compare(res2, oracle.hsvd(G, p, block=B), p)
    assert res2["status"] == 0 and e["sigma_norm"] <= 1e-12 and e["U"] <= 1e-12
    # FP64 only; the pairwise path has no blocks
    assert run_lib(hsvd_ctx, G, p, block=B, precision=H.MIXED)["status"] == H.E_INVAL
    assert run_lib(hsvd_ctx, G, p, block=B, algo=H.PAIRWISE)["status"] == H.E_INVAL
    a = run_lib(hsvd_ctx, G, p, algo=2, block=B)
    b = run_lib(hsvd_ctx, G, p, algo=2, block=B)
    for k in ("sigma", "U", "V", "lam", "perm"):
        assert np.array_equal(a[k], b[k]), k
    assert run_lib(hsvd_ctx, G, p, algo=2, block=B, max_sweeps=1)["status"] == H.E_NOCONV


def test_wide_full_block(hsvd_ctx):
    """The full-block method (Sec. 6) with b = 64: every outer step diagonalises
    its 128-column pivot block."""
    G = W.colscaled(256, 2.0, seed=91)
    p = 100
    ref = oracle.hsvd(G, p, block=B, inner_sweeps=30)
    res = run_lib(hsvd_ctx, G, p, algo=2, block=B, inner_sweeps=30)
    _gate(G, p, res, ref)


@pytest.mark.timeout(900)
def test_wide_colscaled1024(hsvd_ctx):
    G = W.colscaled(1024, 4.0, seed=1001)
    p = 512
    spread, ref = twin_spread(G, p, block=B)
    say("colscaled1024 b=64 twin spread", spread)
    res = run_lib(hsvd_ctx, G, p, algo=2, block=B)
    _gate(G, p, res, ref, uv_gate=max(1e-12, 10 * max(spread["U"], spread["V"])))
