"""Comparison of a library result with the oracle's (several results are correct).

Both results are canonicalised first: within each J class the columns are
ordered by sigma descending; then each library column pair (u_k, v_k) is
flipped so that the entry of u_k at the row where the oracle's u_k is largest
in magnitude has the oracle's sign.  Then sigma is compared normwise and
componentwise, U and V in the Frobenius norm.
"""
from __future__ import annotations

import numpy as np

import oracle


def canon(sig, U, V, p):
    n = sig.size
    pos = sorted(range(p), key=lambda c: -sig[c])
    neg = sorted(range(p, n), key=lambda c: -sig[c])
    o = np.array(pos + neg, dtype=int)
    return sig[o], U[:, o], (V[:, o] if V is not None else None)


def compare(lib_res, orc_res, p):
    """Returns a dict of relative errors of the library result vs the oracle's."""
    s1, U1, V1 = canon(lib_res["sigma"], lib_res["U"], lib_res.get("V"), p)
    s0, U0, V0 = canon(orc_res["sigma"], orc_res["U"], orc_res.get("V"), p)
    n = s0.size
    rows = np.argmax(np.abs(U0), axis=0)
    flip = np.sign(U0[rows, np.arange(n)]) * np.sign(U1[rows, np.arange(n)])
    flip[flip == 0] = 1.0
    U1 = U1 * flip
    out = dict(
        sigma_norm=float(np.linalg.norm(s1 - s0) / np.linalg.norm(s0)),
        sigma_max=float(np.max(np.abs(s1 - s0) / s0)),
        U=float(np.linalg.norm(U1 - U0) / np.linalg.norm(U0)),
    )
    if V0 is not None and V1 is not None:
        V1 = V1 * flip
        out["V"] = float(np.linalg.norm(V1 - V0) / np.linalg.norm(V0))
    return out


def twin_spread(G, p, **kw):
    """Spread between two oracle runs that differ only in summation order:
    the oracle on G and on G with its rows reversed (U's rows un-reversed)."""
    a = oracle.hsvd(G, p, **kw)
    b = oracle.hsvd(np.asfortranarray(G[::-1, :]), p, **kw)
    b = dict(b)
    b["U"] = b["U"][::-1, :]
    return compare(b, a, p), a


def ordering_spread(G, p, **kw):
    """Spread between two oracle runs that follow different trajectories: the
    modified modulus and the round-robin ordering.  The stop rule of eq. (4.2)
    accepts a sweep whose tangents are all at most T, so any two converged
    iterates may differ by the residual off-diagonal level over the spectral
    gaps; a path that takes its own trajectory (the mixed-precision sweeps) is
    gated against this spread, not against the twin spread."""
    a = oracle.hsvd(G, p, ordering="modmod", **kw)
    b = oracle.hsvd(G, p, ordering="roundrobin", **kw)
    return compare(b, a, p), a
