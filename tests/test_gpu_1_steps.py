"""Bit-exact gates of the individual steps on identical inputs (GPU)."""
import numpy as np
import pytest

import oracle
from gpu_util import say

pytestmark = pytest.mark.gpu


def _random_triples(m, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    aii = 10.0 ** g.uniform(-30, 30, m)
    ajj = aii * 10.0 ** g.uniform(-12, 12, m)
    # |a_ij| <= sqrt(a_ii a_jj) (a Gram matrix), with many near-equal / near-parallel cases
    cosang = g.uniform(-1, 1, m) ** g.choice([1, 3, 9], m)
    aij = cosang * np.sqrt(aii) * np.sqrt(ajj)
    eq = g.uniform(size=m) < 0.05
    ajj[eq] = aii[eq]
    tiny = g.uniform(size=m) < 0.05
    aij[tiny] *= 1e-17
    hyp = np.where(g.uniform(size=m) < 0.5, -1, 1).astype(np.int32)
    return aii, ajj, aij, hyp


def test_pair_params_bit_exact(hsvd_ctx):
    import torch

    from paper_1008_1371_amd import hsvd as H
    m = 1_000_000
    aii, ajj, aij, hyp = _random_triples(m, 123)
    edge = np.array([[2.0, 2.0, 0.5, -1], [2.0, 2.0, -0.5, -1], [4.0, 4.0, 4.0, 1],
                     [4.0, 4.0, -4.0, 1], [3.0, 1.0, 1e-200, -1], [3.0, 1.0, 1e-200, 1],
                     [4.0, 4.0, 1.0, -1], [1.0, 1e-300, 1e-151, 1], [1e300, 1e300, 1e299, 1]])
    aii = np.r_[aii, edge[:, 0]]
    ajj = np.r_[ajj, edge[:, 1]]
    aij = np.r_[aij, edge[:, 2]]
    hyp = np.r_[hyp, edge[:, 3].astype(np.int32)]
    tol, T = 1e-13, 0.5e-6
    say("pair_params", aii.size)
    want = oracle.pair_params_batch(aii, ajj, aij, hyp, tol, T)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = H.hsvd_pair_params(hsvd_ctx, dev(aii), dev(ajj), dev(aij), dev(hyp), tol, T)
    for k in ("skip", "status", "code"):
        assert np.array_equal(got[k].cpu().numpy(), want[k]), k
    for k in ("t", "c"):
        g = got[k].cpu().numpy()
        bad = np.flatnonzero(g.view(np.int64) != want[k].view(np.int64))
        assert bad.size == 0, (k, bad[:5], g[bad[:5]], want[k][bad[:5]])


def test_block_pair_params_close(hsvd_ctx):
    """The block path's short-chain rotation vs the oracle's: same skip and rank
    decisions, t and c within a few ulps (times the conditioning of t near
    |t| = 1 for hyperbolic pairs); annihilation checked through the 2x2 data."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    m = 200_000
    aii, ajj, aij, hyp = _random_triples(m, 321)
    tol, T = 1e-13, 0.5e-6
    want = oracle.pair_params_batch(aii, ajj, aij, hyp, tol, T)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = H.hsvd_pair_params(hsvd_ctx, dev(aii), dev(ajj), dev(aij), dev(hyp), tol, T, block=True)
    g = {k: v.cpu().numpy() for k, v in got.items()}
    # decisions at the exact boundary may differ through rounding; none here
    assert np.array_equal(g["skip"], want["skip"])
    live = (want["skip"] == 0) & (want["status"] == 0)
    tie = live & (hyp < 0) & (ajj == aii)
    ok = live & ~tie
    assert np.array_equal(g["status"][live], want["status"][live])
    tw, tg = want["t"][ok], g["t"][ok]
    cond = np.where(hyp[ok] > 0, 1.0 / np.maximum(1e-300, 1 - np.abs(tw)), 1.0)
    assert (np.abs(tg - tw) <= 8 * 2.0 ** -53 * np.abs(tw) * cond).all()
    cw, cg = want["c"][ok], g["c"][ok]
    assert (np.abs(cg - cw) <= 8 * 2.0 ** -53 * cw * cond ** 2).all()
    assert (np.abs(np.abs(g["t"][tie]) - 1.0) <= 4 * 2.0 ** -53).all()


@pytest.mark.parametrize("r", [2, 4, 8, 10, 130, 1024, 4096])
@pytest.mark.parametrize("ordering", ["modmod", "roundrobin"])
def test_pivot_trace_bit_exact(hsvd_ctx, r, ordering):
    from paper_1008_1371_amd import hsvd as H
    steps = 2 * r + 1 if r <= 1024 else r + 1
    say("pivot_trace", ordering, r, steps)
    if ordering == "modmod":
        want = oracle.modmod_trace(r, steps)
        got = H.hsvd_pivot_trace(hsvd_ctx, H.MODMOD, r, steps).cpu().numpy()
    else:
        want = oracle.roundrobin_trace(r, steps)
        got = H.hsvd_pivot_trace(hsvd_ctx, H.ROUNDROBIN, r, steps).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("r,p", [(1, 0), (1, 1), (7, 3), (128, 64), (1000, 0), (1000, 1000),
                                 (4096, 2048), (8194, 3000), (16384, 100)])
def test_sort_bit_exact(hsvd_ctx, r, p):
    import torch

    from paper_1008_1371_amd import hsvd as H
    g = np.random.Generator(np.random.PCG64(r + p))
    d = np.round(g.uniform(0, 8, r) * 4) / 4  # ties
    d[: r // 3] = g.uniform(0, 8, r // 3)
    rho = g.permutation(r).astype(np.int32)
    say("sort", r, p)
    wd, wr = oracle.sort_diag(d, rho, p)
    dd = torch.from_numpy(d.copy()).cuda()
    rr = torch.from_numpy(rho.copy()).cuda()
    H.hsvd_sort_diag(hsvd_ctx, dd, rr, p)
    assert np.array_equal(dd.cpu().numpy(), wd) and np.array_equal(rr.cpu().numpy(), wr)


def _total_order_key(d):
    k = d.view(np.int64)
    return np.where(k < 0, k ^ np.int64(0x7FFFFFFFFFFFFFFF), k)


@pytest.mark.parametrize("r,p", [(64, 20), (1000, 400), (5000, 2500)])
def test_sort_non_finite_keys_give_a_permutation(hsvd_ctx, r, p):
    """NaN, infinities and signed zeros (which the solver never produces):
    the sort still returns a permutation of rho, in the IEEE total order of
    the keys, stable."""
    import torch

    from paper_1008_1371_amd import hsvd as H
    g = np.random.Generator(np.random.PCG64(7 * r + p))
    d = g.uniform(-4, 4, r)
    specials = np.array([np.nan, -np.nan, np.inf, -np.inf, 0.0, -0.0, 1.0, 1.0])
    d[g.integers(0, r, r // 4)] = g.choice(specials, r // 4)
    rho = g.permutation(r).astype(np.int32)
    say("sort non-finite", r, p)
    dd = torch.from_numpy(d.copy()).cuda()
    rr = torch.from_numpy(rho.copy()).cuda()
    H.hsvd_sort_diag(hsvd_ctx, dd, rr, p)
    got_d, got_r = dd.cpu().numpy(), rr.cpu().numpy()
    assert np.array_equal(np.sort(got_r), np.sort(rho))
    key = _total_order_key(d)
    idx = np.arange(r)
    o1 = np.lexsort((idx[:p], ~key[:p]))  # decreasing, ties by position
    o2 = p + np.lexsort((idx[p:], key[p:]))  # increasing
    order = np.concatenate([o1, o2])
    assert np.array_equal(got_r, rho[order])
    assert np.array_equal(got_d.view(np.int64), d[order].view(np.int64))
