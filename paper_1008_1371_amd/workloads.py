"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws matrices and
signatures.  The paper's own test matrices come from an extended-precision
indefinite factorisation that is not available here (Sec. 5); these
generators stand in for them with the shapes of the target workloads:

* ``gaussian``   -- i.i.d. N(0, 1) entries.
* ``colscaled``  -- N(0, 1) times diag(logspace(0, -decades, n)) (condition
                    number about 10**decades set by column scaling).
* ``graded``     -- Q1 diag(logspace(0, -log10(kappa), n)) Q2 with Haar
                    orthogonal Q1, Q2 (QR of a Gaussian with sign-fixed R).
* ``batch``      -- many small Gaussian problems with n_k ~ U{lo..hi} and
                    p_k ~ U{0..n_k}.
* ``indefinite`` -- the paper's own kind of input (Sec. 5): a symmetric
                    indefinite M with a random spectrum, uniform in
                    [-a, -a 1e-5] u [a 1e-5, a] with a from Table 5.2, formed
                    as Q diag(lam) Q^T and factorised M = G J G^T by complete
                    pivoting, both in x87 extended precision (host C,
                    ``csrc/gen_indefinite.c``); G rounded to double.  The
                    spectrum is returned for the eigenvalue errors.
* ``shorten``    -- QR shortening of a tall factor (Sec. 1): HSVD of the
                    square R, left vectors premultiplied by Q.

All draws use numpy's PCG64 with explicit seeds.
"""
from __future__ import annotations

import ctypes
import functools
import os

import numpy as np

SEED_G = 1000
SEED_Q1 = 2000
SEED_Q2 = 3000
SEED_BATCH_SIZES = 4000
SEED_BATCH_G = 5000
SEED_EIG = 6000

GEN_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhsvd_gen.so")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(n: int, seed: int = SEED_G) -> np.ndarray:
    return np.asfortranarray(rng(seed).standard_normal((n, n)))


def colscaled(n: int, decades: float = 4.0, seed: int = SEED_G) -> np.ndarray:
    G = rng(seed).standard_normal((n, n))
    return np.asfortranarray(G * np.logspace(0.0, -decades, n)[None, :])


def haar(n: int, seed: int) -> np.ndarray:
    Q, R = np.linalg.qr(rng(seed).standard_normal((n, n)))
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def graded(n: int, kappa: float, seed1: int = SEED_Q1, seed2: int = SEED_Q2) -> np.ndarray:
    Q1 = haar(n, seed1)
    Q2 = haar(n, seed2)
    s = np.logspace(0.0, -np.log10(kappa), n)
    return np.asfortranarray((Q1 * s[None, :]) @ Q2)


def batch(count: int, lo: int = 8, hi: int = 256, seed_sizes: int = SEED_BATCH_SIZES,
          seed_g: int = SEED_BATCH_G):
    """Returns (ns, ps, Gs): sizes, positive-sign counts and a list of
    Fortran-ordered Gaussian matrices."""
    g = rng(seed_sizes)
    ns = g.integers(lo, hi + 1, size=count)
    ps = np.array([g.integers(0, n + 1) for n in ns])
    Gs = [gaussian(int(n), seed_g + k) for k, n in enumerate(ns)]
    return ns.astype(np.int32), ps.astype(np.int32), Gs


def pack_batch(Gs):
    """Packs column-major matrices back to back; returns (flat, offsets)."""
    offs = np.zeros(len(Gs), dtype=np.int64)
    tot = 0
    for k, G in enumerate(Gs):
        offs[k] = tot
        tot += G.size
    flat = np.empty(tot)
    for k, G in enumerate(Gs):
        flat[offs[k]: offs[k] + G.size] = np.asarray(G).reshape(-1, order="F")
    return flat, offs


def spectrum_bound(n: int) -> float:
    """The bound a of the spectrum for matrix order n (Table 5.2; the last
    value beyond the table)."""
    for limit, a in ((3168, 20.0), (6368, 30.0), (9568, 40.0)):
        if n <= limit:
            return a
    return 50.0


@functools.lru_cache(maxsize=1)
def _gen_lib():
    if not os.path.exists(GEN_LIB):
        raise FileNotFoundError(f"{GEN_LIB} is not built (python -m paper_1008_1371_amd.build)")
    L = ctypes.CDLL(GEN_LIB)
    f = L.hsvd_gen_indefinite
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    return L


@functools.lru_cache(maxsize=4)
def _indefinite(n: int, seed: int, npos, a, nthreads: int):
    g = rng(seed)
    a = spectrum_bound(n) if a is None else float(a)
    mag = g.uniform(a * 1e-5, a, size=n)
    if npos is None:
        sgn = np.where(g.random(n) < 0.5, 1.0, -1.0)
    else:
        sgn = np.concatenate([np.ones(npos), -np.ones(n - npos)])
        g.shuffle(sgn)
    lam = np.ascontiguousarray(mag * sgn)
    vec = np.ascontiguousarray(g.standard_normal((n, n)))
    G = np.empty((n, n), order="F")
    jsig = np.empty(n, dtype=np.int8)
    n2 = ctypes.c_int(0)
    st = _gen_lib().hsvd_gen_indefinite(n, lam.ctypes.data, vec.ctypes.data, int(nthreads), G.ctypes.data,
                                        jsig.ctypes.data, ctypes.byref(n2))
    if st != 0:
        raise RuntimeError(f"hsvd_gen_indefinite({n}) failed: {st}")
    for x in (G, jsig, lam):
        x.setflags(write=False)
    return G, jsig, lam, n2.value


def indefinite(n: int, seed: int = SEED_EIG, npos: int | None = None, a: float | None = None,
               nthreads: int = 0):
    """(G, jsig, lam, blocks2): M = G diag(jsig) G^T has the spectrum lam
    (to extended-precision accuracy before G's rounding).  npos: exact number
    of positive eigenvalues (default: each sign with probability 1/2);
    blocks2: number of 2 x 2 pivots.  Arrays are read-only (cached)."""
    return _indefinite(int(n), int(seed), None if npos is None else int(npos), a, int(nthreads))


def eigen(n: int, seed: int = SEED_EIG, npos: int | None = None, a: float | None = None):
    """(G, p, lam): the factor of ``indefinite`` with its columns stably
    reordered so that the p columns of sign +1 come first (J = diag(I_p,
    -I_{n-p}); a column permutation leaves G J G^T unchanged)."""
    G, jsig, lam, _ = indefinite(n, seed, npos, a)
    order = np.argsort(-jsig.astype(np.int64), kind="stable")
    return np.asfortranarray(G[:, order]), int((jsig > 0).sum()), np.array(lam)


def shorten(G: np.ndarray):
    """QR shortening of a tall factor G (m x n, m >= n): (Q, R) with G = Q R,
    Q m x n with orthonormal columns, R n x n.  The HSVD of R with the same J
    gives the eigenvalues of G J G^T; its left vectors times Q are G's."""
    Q, R = np.linalg.qr(np.asarray(G), mode="reduced")
    return Q, np.asfortranarray(R)


# Named workloads: (generator, n, p) with the sizes the method is measured on.
def workload(name: str):
    """Returns (G, p) for a named workload."""
    if name == "gauss128":
        return gaussian(128), 64
    if name == "graded1024":
        return graded(1024, 1e8), 768
    if name == "graded1024_definite":
        return graded(1024, 1e8), 1024
    if name.startswith("colscaled") and name[9:].isdigit():
        n = int(name[9:])
        return colscaled(n, 4.0), n // 2
    if name.startswith("eigen"):
        # eigen<n>: the paper's test-matrix kind at order n (about equal
        # signs); eigen<n>_p<k>: exactly k positive eigenvalues (Table 5.3)
        body = name[5:]
        npos = int(body.split("_p")[1]) if "_p" in body else None
        G, p, _ = eigen(int(body.split("_p")[0]), npos=npos)
        return G, p
    if name.startswith("graded") and "_k" in name:
        # graded<n>_k<kappa>[_p<p/n>]
        n = int(name[6:name.index("_k")])
        kappa = float(name.split("_k")[1].split("_")[0])
        frac = float(name.split("_p")[1]) if "_p" in name else 0.5
        return graded(n, kappa), int(round(n * frac))
    raise KeyError(name)
