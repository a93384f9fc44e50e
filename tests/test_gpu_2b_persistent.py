"""Persistent pairwise kernel: every sweep of a solve in one cooperative launch,
steps separated per column (persistent = 1) or by a grid barrier
(persistent = 2), the diagonal sort and the stop rule (eq. 4.2) on the device.
It makes the same pair visits in the same order as the per-step launches, so
its results are bit-identical to theirs, whose parity with the oracle the
pairwise tests establish; one case is also gated against the oracle directly
(GPU)."""
import numpy as np
import pytest

import oracle
import pins
from gpu_util import run_lib, say
from parity import compare
from paper_1008_1371_amd import workloads as W

pytestmark = pytest.mark.gpu
MODES = [1, 2]


def _same(res, ref, what):
    assert res["status"] == ref["status"], (what, res["status"], ref["status"])
    for k in ("sweeps", "rotations", "skips", "steps", "code"):
        assert res["info"][k] == ref["info"][k], (what, k, res["info"][k], ref["info"][k])
    for key in ("sigma", "U", "V", "lam", "perm"):
        a, b = res[key], ref[key]
        assert (a is None) == (b is None), (what, key)
        if a is not None:
            assert np.array_equal(a, b), (what, key)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n,p", [(1, 1), (2, 1), (3, 1), (5, 5), (64, 0), (65, 32), (127, 100), (200, 7),
                                 (257, 128), (513, 256)])
def test_persistent_matches_step_launches(hsvd_ctx, mode, n, p):
    G = W.colscaled(n, 2.0, seed=40 + n)
    for ordering in (0, 1):
        say("persistent", mode, "n", n, "p", p, "ordering", ordering)
        ref = run_lib(hsvd_ctx, G, p, algo=1, ordering=ordering)
        res = run_lib(hsvd_ctx, G, p, algo=1, ordering=ordering, persistent=mode)
        _same(res, ref, (n, p, ordering))


@pytest.mark.parametrize("mode", MODES)
def test_persistent_against_oracle(hsvd_ctx, mode):
    G, p = W.workload("gauss128")
    say("persistent gauss128 vs oracle", mode)
    ref = oracle.hsvd(G, p)
    res = run_lib(hsvd_ctx, G, p, algo=1, persistent=mode)
    assert res["status"] == 0
    e = compare(res, ref, p)
    say("   errors", e, "sweeps lib/orc", res["info"]["sweeps"], ref["sweeps"])
    assert res["info"]["sweeps"] == ref["sweeps"]
    assert e["sigma_norm"] <= 1e-12 and e["U"] <= 1e-12 and e["V"] <= 1e-12, e
    pins.check_invariants(G, p, res, tol=ref["tol"])


@pytest.mark.parametrize("mode", MODES)
def test_persistent_options_and_stops(hsvd_ctx, mode):
    """Unsorted, without V, stopped by max_sweeps after 1 .. 3 sweeps (the
    state returned after each is the per-step path's), and rank deficiency
    found inside a sweep (same sweep, same status)."""
    from paper_1008_1371_amd import hsvd as H
    G = W.graded(256, 1e6, seed1=71, seed2=72)
    for kw in (dict(sort=0), dict(want_v=0), dict(max_sweeps=1), dict(max_sweeps=2), dict(max_sweeps=3),
               dict(ordering=1, max_sweeps=2)):
        say("persistent options", mode, kw)
        ref = run_lib(hsvd_ctx, G, 160, algo=1, **kw)
        res = run_lib(hsvd_ctx, G, 160, algo=1, persistent=mode, **kw)
        _same(res, ref, kw)
    assert run_lib(hsvd_ctx, G, 160, algo=1, persistent=mode, max_sweeps=1)["status"] == H.E_NOCONV
    g = W.gaussian(16, seed=3)
    gd = g.copy()
    gd[:, 12] = gd[:, 3]
    gz = g.copy()
    gz[:, 5] = 0.0
    for what, M, kw in (("duplicate column", gd, dict(sort=0)), ("zero column", gz, {})):
        say("persistent rank", mode, what)
        ref = run_lib(hsvd_ctx, M, 8, algo=1, **kw)
        res = run_lib(hsvd_ctx, M, 8, algo=1, persistent=mode, **kw)
        assert res["status"] == ref["status"] == H.E_RANK, (what, res["status"])
    assert run_lib(hsvd_ctx, g, 8, algo=1, persistent=3)["status"] == H.E_INVAL
    D = np.diag(np.arange(1.0, 17.0))
    R = run_lib(hsvd_ctx, D, 5, algo=1, persistent=mode)
    assert R["status"] == 0 and R["info"]["sweeps"] == 1 and R["info"]["rotations"] == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,p", [("graded1024", 768), ("colscaled4096", 2048)])
def test_persistent_full_size(hsvd_ctx, name, p):
    """The pairwise workloads at full size: graded n = 1024 (one slot per
    workgroup) and colscaled n = 4096 (2048 slots on fewer resident
    workgroups, each visiting several slots per step)."""
    G, _ = W.workload(name)
    ref = run_lib(hsvd_ctx, G, p, algo=1)
    for mode in MODES:
        res = run_lib(hsvd_ctx, G, p, algo=1, persistent=mode)
        say("persistent", name, mode, "sweeps", res["info"]["sweeps"], "ms", res["info"]["ms_total"], "steps ms",
            ref["info"]["ms_total"])
        _same(res, ref, (name, mode))
