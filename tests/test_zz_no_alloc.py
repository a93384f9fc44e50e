"""hsvd_solve_noalloc (the entry point that allocates no device memory) against
hsvd_solve on the same inputs, through the C ABI (GPU).

Both entry points run the same kernels with the same launch shapes; only the
workspace differs (the library's fixed scratch array instead of its grown
workspace).  Each case makes two noalloc calls in a row, the second with a
smaller input, so the second call runs on what the first left in the scratch
array.  Gate: sigma normwise and U, V in the Frobenius norm within 1e-12 of
hsvd_solve's result (the parity bar); the test also reports whether the two
results are bit-identical.
"""
import numpy as np
import pytest

from gpu_util import say, to_dev
from paper_1008_1371_amd import hsvd as H
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # (label, params, (n1, p1), (n2, p2))
    ("pairwise fp64", dict(algo=H.PAIRWISE), (300, 120), (97, 50)),
    ("block fp64", dict(algo=H.BLOCK), (640, 320), (200, 77)),
    ("mixed", dict(algo=H.BLOCK, precision=H.MIXED), (1024, 512), (384, 100)),
]


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def _pair(ctx, G, p, prm):
    Gt = to_dev(G)
    ref = H.hsvd_solve(ctx, Gt, p, prm, check=False)
    got = H.hsvd_solve_noalloc(ctx, Gt, p, prm, check=False)
    return ref, got


@pytest.mark.parametrize("label,kw,first,second", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_solve(hsvd_ctx, label, kw, first, second):
    prm = H.hsvd_default_params(**kw)
    inputs = [(n, p, to_dev(W.colscaled(n, 2.0, seed=900 + n))) for n, p in (first, second)]
    refs = [H.hsvd_solve(hsvd_ctx, Gt, p, prm, check=False) for n, p, Gt in inputs]
    # the two noalloc calls back to back, the second on the smaller input
    gots = []
    for call, (n, p, Gt) in enumerate(inputs):
        say("noalloc", label, "call", call, "n", n, "p", p)
        gots.append(H.hsvd_solve_noalloc(hsvd_ctx, Gt, p, prm, check=False))
    for call, ((n, p, _), ref, got) in enumerate(zip(inputs, refs, gots)):
        assert ref["status"] == H.OK and got["status"] == H.OK, (ref["status"], got["status"])
        ri, gi = ref["info"], got["info"]
        assert (gi["sweeps"], gi["sweeps_fp32"], gi["r"], gi["block"], gi["ldg"]) == \
            (ri["sweeps"], ri["sweeps_fp32"], ri["r"], ri["block"], ri["ldg"])
        assert gi["ms_total"] == 0.0
        errs = {}
        same = True
        for k in ("sigma", "U", "V", "lam"):
            a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
            errs[k] = _rel(a, b)
            same = same and np.array_equal(a, b)
        same = same and np.array_equal(got["perm"].cpu().numpy(), ref["perm"].cpu().numpy())
        say("   sweeps", gi["sweeps_fp32"], gi["sweeps"], "rel diffs", errs, "bit-identical", same)
        assert errs["sigma"] <= 1e-12 and errs["lam"] <= 1e-12, errs
        assert errs["U"] <= 1e-12 and errs["V"] <= 1e-12, errs


def test_noalloc_rejects_what_does_not_fit(hsvd_ctx):
    """A solve whose workspace exceeds the scratch array returns E_SIZE before
    any launch, and the next call that fits still works."""
    import torch
    n = 2048
    G = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    R = H.hsvd_solve_noalloc(hsvd_ctx, G, n // 2, H.hsvd_default_params(precision=H.MIXED), check=False)
    assert R["status"] == H.E_SIZE
    # the persistent pairwise kernel (a cooperative launch) is not offered here
    R = H.hsvd_solve_noalloc(hsvd_ctx, G[:64, :64].contiguous(), 32,
                             H.hsvd_default_params(algo=H.PAIRWISE, persistent=1), check=False)
    assert R["status"] == H.E_INVAL
    Gs = W.gaussian(64, seed=5)
    ref, got = _pair(hsvd_ctx, Gs, 32, H.hsvd_default_params())
    assert got["status"] == H.OK
    assert _rel(got["sigma"].cpu().numpy(), ref["sigma"].cpu().numpy()) <= 1e-12
