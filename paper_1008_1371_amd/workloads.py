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

All draws use numpy's PCG64 with explicit seeds.
"""
from __future__ import annotations

import numpy as np

SEED_G = 1000
SEED_Q1 = 2000
SEED_Q2 = 3000
SEED_BATCH_SIZES = 4000
SEED_BATCH_G = 5000


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


# Named workloads: (generator, n, p) with the sizes the method is measured on.
def workload(name: str):
    """Returns (G, p) for a named workload."""
    if name == "gauss128":
        return gaussian(128), 64
    if name == "graded1024":
        return graded(1024, 1e8), 768
    if name == "graded1024_definite":
        return graded(1024, 1e8), 1024
    if name == "colscaled4096":
        return colscaled(4096, 4.0), 2048
    if name.startswith("graded4096_k"):
        kappa = float(name.split("_k")[1].split("_")[0])
        frac = float(name.split("_p")[1]) if "_p" in name else 0.5
        return graded(4096, kappa), int(round(4096 * frac))
    raise KeyError(name)
