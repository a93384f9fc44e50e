"""Whole-solve properties of the oracle (CPU only)."""
import numpy as np
import pytest

import oracle
import pins
from paper_1008_1371_amd import workloads as W


def test_threads_bit_identical():
    G = W.colscaled(96, 3.0, seed=17)
    a = oracle.hsvd(G, 40, nthreads=1)
    b = oracle.hsvd(G, 40, nthreads=4)
    for k in ("sigma", "U", "V", "lam", "perm"):
        assert np.array_equal(a[k], b[k]), k
    a = oracle.hsvd(G, 40, block=8, nthreads=1)
    b = oracle.hsvd(G, 40, block=8, nthreads=4)
    for k in ("sigma", "U", "V", "lam", "perm"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("mode", [dict(ordering="roundrobin"), dict(block=4), dict(block=16),
                                  dict(sort=False), dict(ordering="roundrobin", block=8)])
def test_orderings_agree(mode):
    G = W.gaussian(64, seed=21)
    ref = oracle.hsvd(G, 30)
    R = oracle.hsvd(G, 30, **mode)
    assert R["status"] == 0
    pins.check_invariants(G, 30, R, tol=R["tol"])
    a = np.sort(ref["lam"])
    b = np.sort(R["lam"])
    assert np.linalg.norm(a - b) / np.linalg.norm(a) <= 1e-14


def test_bordering_matches_explicit_border():
    """An odd order is bordered by a unit column with a negative sign (eq. 4.1):
    solving the bordered matrix explicitly gives bit-identical results."""
    n, p = 31, 12
    G = W.gaussian(n, seed=8)
    Gb = np.zeros((n + 1, n + 1), order="F")
    Gb[:n, :n] = G
    Gb[n, n] = 1.0
    a = oracle.hsvd(G, p)
    b = oracle.hsvd(Gb, p)
    assert a["status"] == b["status"] == 0
    assert np.array_equal(a["sigma"], b["sigma"][:n])
    assert np.array_equal(a["U"], b["U"][:n, :n])
    assert np.array_equal(a["V"], b["V"][:n, :n])
    assert a["sweeps"] == b["sweeps"] and a["rotations"] == b["rotations"]


def test_max_steps_sample_stops():
    G = W.gaussian(64, seed=2)
    R = oracle.hsvd(G, 32, max_steps=10)
    assert R["steps"] == 10 and R["status"] == oracle.E_NOCONV


def test_graded_definite_and_indefinite_small():
    G = W.graded(96, 1e8, seed1=5, seed2=6)
    for p in (96, 72):
        R = oracle.hsvd(G, p)
        assert R["status"] == 0
        pins.check_invariants(G, p, R, tol=R["tol"])


def _pair_offdiag(U, cols):
    """Largest |cos| between distinct columns of U in `cols`."""
    Up = U[:, cols]
    C = Up.T @ Up
    return np.max(np.abs(C - np.diag(np.diag(C))))


def test_full_block_diagonalises_each_pivot_block():
    """Full-block mode (Sec. 6): after one outer step every pivot block pair of
    that step is diagonal -- its 2b columns are mutually orthogonal to the skip
    tolerance -- while a single pass over the block pair's pairs (the first
    outer step of the block-oriented method) leaves larger cosines."""
    n, p, b = 128, 64, 32
    G = W.gaussian(n, seed=33)
    # modified modulus over nb = 4 blocks starts on the antidiagonal: (0, 3), (1, 2)
    groups = [np.r_[0:32, 96:128], np.r_[32:96]]
    full = oracle.hsvd(G, p, block=b, sort=False, max_steps=1, inner_sweeps=30)
    once = oracle.hsvd(G, p, block=b, sort=False, max_steps=1)
    assert full["status"] == once["status"] == oracle.E_NOCONV
    tol = full["tol"]
    for cols in groups:
        assert _pair_offdiag(full["U"], cols) <= 2 * tol
    assert max(_pair_offdiag(once["U"], c) for c in groups) > 100 * tol
    assert full["inner"] > 2 * 2  # several inner sweeps per block pair, two pairs


def test_full_block_solution():
    """The full-block oracle converges to the same decomposition, in fewer outer
    sweeps and with more rotations than the block-oriented one."""
    G = W.colscaled(192, 3.0, seed=34)
    p = 80
    full = oracle.hsvd(G, p, block=32, inner_sweeps=30)
    once = oracle.hsvd(G, p, block=32)
    assert full["status"] == once["status"] == 0
    pins.check_invariants(G, p, full, tol=full["tol"])
    assert full["sweeps"] < once["sweeps"] and full["rotations"] > once["rotations"]
    # both within the eigenvalue invariant's ~10 n u of eig(G J G^T)
    a, c = np.sort(full["lam"]), np.sort(once["lam"])
    assert np.linalg.norm(a - c) / np.linalg.norm(c) <= 20 * 192 * 2.0 ** -53
    # inner_sweeps = 1 is a single pass over all pairs in every outer step
    one = oracle.hsvd(G, p, block=32, inner_sweeps=1)
    assert one["status"] == 0 and one["inner"] == one["steps"] * (one["r"] // 32 // 2)
