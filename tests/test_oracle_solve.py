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
