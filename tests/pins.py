"""Pins for the oracle: checks against what the paper and the mathematics fix.

Each function raises AssertionError when the oracle (the module ``oracle``,
whose loaded library may be swapped for a planted-mistake build) disagrees
with an independent fact:

* the defining property of a Jacobi rotation -- a'_ij = 0 after the update
  rules (2.4)/(2.5) -- evaluated in 50-digit arithmetic, plus the diagonal
  identities (2.6) and cos/cosh relations of (2.2);
* t against the tangent of half of atan / atanh of the exact 2x2 data;
* the convergence code table of (4.2) and the strict inequality of (2.3);
* the modified modulus strategy against Sec. 2 (antidiagonal start, r steps,
  (i, q+i) twice, reversed assignment in the next quasi-sweep) and against
  the antidiagonal strategy of the Appendix (Table A.1, golden file);
* the stable diagonal sort against Python's stable ``sorted``;
* J = I against LAPACK's SVD (numpy.linalg.svd) and a symmetric eigensolver
  of G^T G;
* the HSVD invariants U^T U = I, V^T J V = J, G V = U Sigma and the
  eigenvalues of G J G^T (LAPACK eigvalsh, and mpmath at 50 digits on tiny
  inputs).
"""
from __future__ import annotations

import os
from collections import Counter

import mpmath as mp
import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS = 2.0 ** -52
U_RND = 2.0 ** -53


# --------------------------------------------------------------------------
# 2x2 rotation
# --------------------------------------------------------------------------

def _random_pairs(seed, count, hyp):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        m = int(g.integers(2, 9))
        gi = g.standard_normal(m) * 10.0 ** g.uniform(-4, 4)
        gj = g.standard_normal(m) * 10.0 ** g.uniform(-4, 4)
        if g.uniform() < 0.3:
            gj = gj * 1e-3 + gi * g.uniform(-2, 2)
        out.append((gi, gj))
    return out


def _mp_gram(gi, gj):
    gi = [mp.mpf(float(x)) for x in gi]
    gj = [mp.mpf(float(x)) for x in gj]
    return (mp.fsum(x * x for x in gi), mp.fsum(y * y for y in gj),
            mp.fsum(x * y for x, y in zip(gi, gj)), gi, gj)


def pin_rotation_annihilates(count=150):
    """(t, c) from the oracle, applied by (2.4)/(2.5) in 50-digit arithmetic,
    leave a'_ij at rounding level and satisfy (2.6) and c^2 (1 -+ t^2) = 1."""
    with mp.workdps(50):
        for hyp in (-1, 1):
            for gi, gj in _random_pairs(11 + hyp, count, hyp):
                aii = float(np.dot(gi, gi))
                ajj = float(np.dot(gj, gj))
                aij = float(np.dot(gi, gj))
                st, t, c = oracle.rotation(aii, ajj, aij, hyp)
                if hyp > 0 and abs(2 * aij) >= (aii + ajj) * (1 - 1e-12):
                    continue
                assert st == 0, (hyp, aii, ajj, aij)
                assert abs(t) <= 1.0
                # the 2x2 data taken exactly as the doubles given to the oracle
                Aii, Ajj, Aij = mp.mpf(aii), mp.mpf(ajj), mp.mpf(aij)
                T, C = mp.mpf(t), mp.mpf(c)
                # A' = R^T A R, R = [[1, t], [hyp t, 1]] * c  (columns (2.4)/(2.5))
                ht = hyp * T
                a_ij_new = C * C * ((Aii * T) + Aij * (1 + ht * T) + ht * Ajj)
                a_ii_new = C * C * (Aii + 2 * ht * Aij + ht * ht * Ajj)
                a_jj_new = C * C * (T * T * Aii + 2 * T * Aij + Ajj)
                scale = mp.sqrt(Aii * Ajj)
                assert abs(a_ij_new) <= 64 * U_RND * scale / (1 - abs(T)) ** (1 if hyp > 0 else 0), \
                    ("a'_ij not annihilated", hyp, float(a_ij_new / scale))
                # eq. (2.6): a'_ii = a_ii + hyp t a_ij, a'_jj = a_jj + t a_ij
                bound = 64 * U_RND * (Aii + Ajj) / ((1 - T * T) if hyp > 0 else 1)
                assert abs(a_ii_new - (Aii + ht * Aij)) <= bound
                assert abs(a_jj_new - (Ajj + T * Aij)) <= bound
                # eq. (2.2): cos^2 (1 + tan^2) = 1, cosh^2 (1 - tanh^2) = 1
                rel = C * C * (1 + T * T) - 1 if hyp < 0 else C * C * (1 - T * T) - 1
                assert abs(rel) <= 8 * U_RND / ((1 - abs(T)) if hyp > 0 else 1)


def pin_rotation_vs_inverse_functions(count=150):
    """t is tan (tanh) of half the angle whose tan 2phi (tanh 2phi) the 2x2
    data fix, computed here through atan / atanh at 50 digits."""
    with mp.workdps(50):
        for hyp in (-1, 1):
            for gi, gj in _random_pairs(23 + hyp, count, hyp):
                aii = float(np.dot(gi, gi))
                ajj = float(np.dot(gj, gj))
                aij = float(np.dot(gi, gj))
                if aij == 0.0:
                    continue
                Aii, Ajj, Aij = mp.mpf(aii), mp.mpf(ajj), mp.mpf(aij)
                if hyp < 0:
                    if Ajj == Aii:
                        phi = mp.pi / 4 * mp.sign(Aij)
                    else:
                        phi = mp.atan(2 * Aij / (Ajj - Aii)) / 2
                    texact = mp.tan(phi)
                    cexact = mp.cos(phi)
                else:
                    x = -2 * Aij / (Aii + Ajj)
                    if abs(x) >= 1 - mp.mpf(10) ** -12:
                        continue
                    phi = mp.atanh(x) / 2
                    texact = mp.tanh(phi)
                    cexact = mp.cosh(phi)
                st, t, c = oracle.rotation(aii, ajj, aij, hyp)
                assert st == 0
                # relative error of t: a few roundings, amplified by the
                # conditioning of zeta -> t near |t| = 1 for the hyperbolic case
                cond = 1 if hyp < 0 else 1 / (1 - abs(texact))
                assert abs(mp.mpf(t) - texact) <= 16 * U_RND * abs(texact) * cond, \
                    (hyp, t, float(texact))
                assert abs(mp.mpf(c) - cexact) <= 16 * U_RND * cexact * cond * cond


def pin_rotation_edges():
    # equal diagonal, trigonometric: tan 2phi = inf -> phi = pi/4 (sgn(0) = +1)
    st, t, c = oracle.rotation(2.0, 2.0, 0.5, -1)
    assert st == 0 and t == 1.0 and abs(c - 2 ** -0.5) <= 2 ** -53
    # negative a_ij with equal diagonal: zeta = -0.0 counts as +1 (t = +1)
    st, t, c = oracle.rotation(2.0, 2.0, -0.5, -1)
    assert st == 0 and abs(t) == 1.0
    # tiny a_ij: t ~ a_ij / (a_jj - a_ii) (first order), both signs
    for hyp in (-1, 1):
        aii, ajj, aij = 3.0, 1.0, 1e-200
        st, t, c = oracle.rotation(aii, ajj, aij, hyp)
        expect = aij / (ajj - aii) if hyp < 0 else -aij / (aii + ajj)
        assert st == 0 and abs(t - expect) <= 4 * U_RND * abs(expect) and c == 1.0
    # hyperbolic pair of parallel columns of equal norm: |zeta| = 1, rank failure
    st, t, c = oracle.rotation(4.0, 4.0, 4.0, 1)
    assert st == 1
    st, t, c = oracle.rotation(4.0, 4.0, -4.0, 1)
    assert st == 1
    # trigonometric pair of parallel columns is fine (pi/4)
    st, t, c = oracle.rotation(4.0, 4.0, 4.0, -1)
    assert st == 0 and t == 1.0


def pin_skip_and_code():
    # eq. (2.3) is a strict inequality; sqrt(4) sqrt(4) = 4 and 0.25 * 4 = 1 exactly
    assert oracle.skip(4.0, 4.0, 1.0, 0.25) is False
    assert oracle.skip(4.0, 4.0, np.nextafter(1.0, 0.0), 0.25) is True
    assert oracle.skip(4.0, 4.0, -np.nextafter(1.0, 0.0), 0.25) is True
    assert oracle.skip(4.0, 4.0, 0.0, 1e-300) is True
    # eq. (4.2)
    T = 0.1
    for code in (0, 1, 3):
        assert oracle.conv_code(code, 0, 0.5, T) == code
        assert oracle.conv_code(code, 1, 0.5, T) == 3
        assert oracle.conv_code(code, 1, -0.5, T) == 3
        assert oracle.conv_code(code, 1, 0.1, T) == (code | 1)
        assert oracle.conv_code(code, 1, -0.05, T) == (code | 1)


# --------------------------------------------------------------------------
# orderings
# --------------------------------------------------------------------------

def _is_matching(pairs, r):
    flat = np.asarray(pairs).reshape(-1)
    return sorted(flat.tolist()) == list(range(r)) and bool((pairs[:, 0] < pairs[:, 1]).all())


def load_antidiagonal(path=os.path.join(GOLDEN, "antidiagonal_n8.txt")):
    steps = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, rest = line.split(":")
        pairs = []
        for tok in rest.split():
            a, b = tok.strip("()").split(",")
            pairs.append((int(a), int(b)))
        steps[int(k)] = pairs
    return steps


def pin_modmod(rs=(2, 4, 6, 8, 10, 16, 34, 128, 256, 1024)):
    for r in rs:
        q = r // 2
        T = oracle.modmod_trace(r, 2 * r + 1)
        # antidiagonal start (Alg. 4.3)
        assert [tuple(x) for x in T[0]] == [(k, r - 1 - k) for k in range(q)]
        for s in range(2 * r + 1):
            assert _is_matching(T[s], r), (r, s)
        # a quasi-sweep is r steps; every pair once, (i, q+i) twice (Sec. 2)
        for w in (0, 1):
            C = Counter(map(tuple, T[w * r:(w + 1) * r].reshape(-1, 2)))
            assert len(C) == r * (r - 1) // 2
            for (i, j), c in C.items():
                assert c == (2 if j - i == q else 1), (r, i, j, c)
        # the next quasi-sweep starts with the assignment to tasks reversed
        assert (T[r] == T[0][::-1]).all()
        assert (T[2 * r] == T[0]).all()


def pin_modmod_vs_appendix():
    """The modulus strategy's steps are the antidiagonal strategy's steps in
    the order O' of the Appendix: n-1, n, {n+1, 1}, {n+2, 2}, ...,
    {2n-3, n-3}, {n-2} (1-based); the modified strategy adds only pairs
    (i, q+i)."""
    anti = load_antidiagonal()
    n = 8
    assert len(anti) == 2 * n - 3
    order = [[n - 1], [n]] + [[n + k, k] for k in range(1, n - 2)] + [[n - 2]]
    assert len(order) == n
    T = oracle.modmod_trace(n, n)
    for s, group in enumerate(order):
        want = set()
        for m in group:
            want |= {(i - 1, j - 1) for (i, j) in anti[m]}
        got = set(map(tuple, T[s].tolist()))
        assert want <= got, (s, want, got)
        assert all(j - i == n // 2 for (i, j) in got - want), (s, got - want)
    # the same structure at larger r, from the rule of Table A.1
    for r in (16, 64, 256):
        T = oracle.modmod_trace(r, r)
        for s in range(r):
            sums = {r - 1} if s == 0 else {r} if s == 1 else {r - 2} if s == r - 1 else {r - 1 + s, s - 1}
            got = set(map(tuple, T[s].tolist()))
            want = {(i, j) for i in range(r) for j in range(i + 1, r) if i + j in sums}
            assert want <= got and all(j - i == r // 2 for (i, j) in got - want)


def pin_roundrobin(rs=(2, 4, 8, 10, 34, 128, 256)):
    for r in rs:
        T = oracle.roundrobin_trace(r, r - 1)
        # the circle starts in natural order, i.e. on the antidiagonal that
        # Alg. 4.3 also starts from
        assert [tuple(x) for x in T[0]] == [(k, r - 1 - k) for k in range(r // 2)]
        for s in range(r - 1):
            assert _is_matching(T[s], r)
        C = Counter(map(tuple, T.reshape(-1, 2)))
        assert len(C) == r * (r - 1) // 2 and max(C.values()) == 1


def pin_block_ordering(r=32, b=4):
    nb = r // b
    outer = oracle.modmod_trace(nb, nb)
    seen = Counter()
    for s in range(nb):
        pairs = oracle.block_step_pairs(r, b, outer[s], s)
        per = len(pairs) // (nb // 2)
        for k, (I, J) in enumerate(outer[s]):
            blk = pairs[k * per:(k + 1) * per]
            cols = set(range(I * b, I * b + b)) | set(range(J * b, J * b + b))
            assert set(blk.reshape(-1).tolist()) <= cols
            if s == 0:
                want = {(i, j) for i in cols for j in cols if i < j}
                assert len(blk) == len(want) and set(map(tuple, blk.tolist())) == want
                inner = 2 * b - 1
            else:
                want = {(i, j) for i in range(I * b, I * b + b) for j in range(J * b, J * b + b)}
                assert len(blk) == b * b and set(map(tuple, blk.tolist())) == want
                inner = b
            for u in range(inner):
                chunk = blk[u * b:(u + 1) * b]
                assert len(set(chunk.reshape(-1).tolist())) == 2 * b
        seen.update(map(tuple, pairs.tolist()))
    assert len(seen) == r * (r - 1) // 2


# --------------------------------------------------------------------------
# sort
# --------------------------------------------------------------------------

def pin_sort(seed=5):
    g = np.random.Generator(np.random.PCG64(seed))
    for r, p in ((10, 4), (33, 0), (33, 33), (64, 17), (200, 100)):
        d = np.round(g.uniform(0, 4, r) * 2) / 2  # many ties
        rho = g.permutation(r).astype(np.int32)
        ds, rs = oracle.sort_diag(d, rho, p)
        pos = sorted(range(p), key=lambda q: -d[q])
        neg = sorted(range(p, r), key=lambda q: d[q])
        want = pos + neg
        assert (ds == d[want]).all() and (rs == rho[want]).all()


# --------------------------------------------------------------------------
# whole solve
# --------------------------------------------------------------------------

def _canon(U, s, V=None):
    """Columns sorted by sigma descending, signs fixed by U's largest entry."""
    o = np.argsort(-s, kind="stable")
    U = U[:, o].copy()
    s = s[o]
    V = V[:, o].copy() if V is not None else None
    idx = np.argmax(np.abs(U), axis=0)
    sg = np.sign(U[idx, np.arange(U.shape[1])])
    U *= sg
    if V is not None:
        V *= sg
    return U, s, V


def pin_identity_svd(n=48, seed=7):
    g = np.random.Generator(np.random.PCG64(seed))
    G = g.standard_normal((n, n))
    R = oracle.hsvd(G, n)
    assert R["status"] == 0
    Ul, sl, Vlt = np.linalg.svd(G)
    Uc, sc, Vc = _canon(R["U"], R["sigma"], R["V"])
    assert np.max(np.abs(sc - sl) / sl) <= 1e-12 * np.linalg.cond(G) / 100 + 1e-13
    sg = np.sign(Ul[np.argmax(np.abs(Ul), axis=0), np.arange(n)])
    Ul = Ul * sg
    Vl = Vlt.T * sg
    gaps = np.min(np.abs(sl[:, None] - sl[None, :]) + np.eye(n) * 1e9, axis=1) / sl[0]
    assert np.linalg.norm(Uc - Ul) <= 1e-13 / gaps.min() * n
    assert np.linalg.norm(Vc - Vl) <= 1e-13 / gaps.min() * n
    # a separate symmetric eigensolver of G^T G (relative accuracy limited by squaring)
    ev = np.sort(np.linalg.eigvalsh(G.T @ G))[::-1]
    assert np.linalg.norm(sc ** 2 - ev) <= 1e-13 * np.linalg.norm(ev) * np.linalg.cond(G)
    assert np.allclose(R["lam"], R["sigma"] ** 2, rtol=4 * EPS, atol=0)


def check_invariants(G, p, R, *, tol):
    n = G.shape[0]
    U, s, V, lam = R["U"], R["sigma"], R["V"], R["lam"]
    j = np.r_[np.ones(p), -np.ones(n - p)]
    J = np.diag(j)
    UtU = U.T @ U
    off = np.max(np.abs(UtU - np.diag(np.diag(UtU))))
    assert off <= 2 * tol, ("U^T U off-diagonal", off, tol)
    assert np.max(np.abs(np.diag(UtU) - 1)) <= 8 * n * U_RND
    if V is not None:
        vn = np.linalg.norm(V, 2) ** 2
        # each column takes ~n rotations per sweep; their rounding errors add up
        # like a random walk over the n*sweeps rotations, over n^2 entries
        bound = 4 * n * np.sqrt(n * max(R["sweeps"], 1)) * U_RND
        assert np.linalg.norm(V.T @ J @ V - J) / vn <= bound, \
            ("V^T J V", np.linalg.norm(V.T @ J @ V - J) / vn, bound)
        r = np.linalg.norm(G @ V - U * s) / (np.linalg.norm(G) * max(1.0, np.linalg.norm(V, 2)))
        assert r <= 10 * np.sqrt(n) * U_RND, ("G V - U S", r)
    ev = np.sort(np.linalg.eigvalsh(G @ J @ G.T))
    e = np.linalg.norm(np.sort(lam) - ev) / np.linalg.norm(ev)
    # rounding of the rotations applied to each column, accumulated like a
    # random walk: sqrt(rotations per column) u per column, normwise over n
    # (10 n u covers the pointwise and block-oriented methods; the full-block
    # method applies several times more rotations per column)
    rot = R.get("rotations", R.get("info", {}).get("rotations", 0)) or 0
    ebound = max(10 * n * U_RND, 0.5 * np.sqrt(rot / n) * n * U_RND)
    assert e <= ebound, ("eig(G J G^T)", e, ebound)
    # lambda = sigma^2 j: the sign of each physical column's eigenvalue is its J sign
    assert ((lam > 0) == (np.arange(n) < p)).all()
    assert np.allclose(np.abs(lam), s ** 2, rtol=4 * EPS, atol=0)


def pin_invariants(cases=((40, 20), (41, 13), (64, 0), (33, 33))):
    g = np.random.Generator(np.random.PCG64(99))
    for n, p in cases:
        G = g.standard_normal((n, n)) * np.logspace(0, -2, n)[None, :]
        R = oracle.hsvd(G, p)
        assert R["status"] == 0, R["status"]
        check_invariants(G, p, R, tol=R["tol"])


def pin_mpmath_tiny(cases=((4, 2), (6, 1), (7, 4), (9, 9), (12, 5))):
    """Eigenvalues and eigenvectors of M = G J G^T at 50 digits (mpmath
    eigsy) against lambda = sigma^2 j and U."""
    g = np.random.Generator(np.random.PCG64(31))
    with mp.workdps(50):
        for n, p in cases:
            G = g.standard_normal((n, n))
            R = oracle.hsvd(G, p)
            assert R["status"] == 0
            Gm = mp.matrix(G.tolist())
            Jm = mp.diag([1] * p + [-1] * (n - p))
            M = Gm * Jm * Gm.T
            E, Q = mp.eigsy(M)
            ev = np.array([float(E[k]) for k in range(n)])
            o = np.argsort(ev)
            lam = R["lam"]
            ol = np.argsort(lam)
            rel = np.abs(lam[ol] - ev[o]) / np.abs(ev[o])
            assert rel.max() <= 1e-13 * n, (n, p, rel.max())
            Qn = np.array([[float(Q[a, b]) for b in range(n)] for a in range(n)])[:, o]
            Un = R["U"][:, ol]
            for k in range(n):
                c = abs(float(np.dot(Qn[:, k], Un[:, k])))
                gap = np.min(np.abs(np.delete(ev[o], k) - ev[o][k])) / abs(ev[o][k])
                assert 1 - c <= 1e-12 / min(gap, 1) ** 2, (n, p, k, 1 - c)


def pin_stop_and_errors():
    g = np.random.Generator(np.random.PCG64(3))
    G = g.standard_normal((16, 16))
    assert oracle.hsvd(G, 8, max_sweeps=1)["status"] == oracle.E_NOCONV
    # already orthogonal columns: one sweep, no rotation, code 00
    D = np.diag(np.arange(1.0, 17.0))
    R = oracle.hsvd(D, 5)
    assert R["status"] == 0 and R["sweeps"] == 1 and R["code"] == 0 and R["rotations"] == 0
    assert np.allclose(np.sort(R["sigma"]), np.arange(1.0, 17.0), rtol=0, atol=0)
    # duplicate column of opposite sign class, met in the first step (antidiagonal
    # pair (3, 12) without sorting): hyperbolic pair with |zeta| = 1
    Gd = G.copy()
    Gd[:, 12] = Gd[:, 3]
    assert oracle.hsvd(Gd, 8, sort=False)["status"] == oracle.E_RANK
    Gz = G.copy()
    Gz[:, 5] = 0.0
    assert oracle.hsvd(Gz, 8)["status"] == oracle.E_RANK
    Gn = G.copy()
    Gn[2, 2] = np.nan
    assert oracle.hsvd(Gn, 8)["status"] == oracle.E_INVAL
    assert oracle.hsvd(G, 17)["status"] == oracle.E_INVAL
    assert oracle.hsvd(G, -1)["status"] == oracle.E_INVAL


ALL_PINS = [pin_rotation_annihilates, pin_rotation_vs_inverse_functions, pin_rotation_edges,
            pin_skip_and_code, pin_modmod, pin_modmod_vs_appendix, pin_roundrobin,
            pin_block_ordering, pin_sort, pin_identity_svd, pin_invariants, pin_mpmath_tiny,
            pin_stop_and_errors]
