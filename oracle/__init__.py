"""Oracle for the one-sided Jacobi hyperbolic SVD (plain FP64 C on the CPU).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the library never
does.  It shares no code with the HIP library: its arithmetic lives in
``hsvd_oracle.c`` (Novakovic & Singer, Secs. 2 and 4, eqs. 2.2-2.6, 4.1, 4.2,
Algs. 4.1-4.5) and this module only marshals NumPy arrays through ctypes.

Parity pins (closed forms, LAPACK SVD for J = I, eigenvalues of G J G^T in
50-digit arithmetic, stepper properties from Sec. 2 and the Appendix) live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hsvd_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

OK, E_INVAL, E_NOCONV, E_RANK = 0, -1, -2, -3
MODMOD, ROUNDROBIN = 0, 1


def build() -> str:
    """Compile the oracle with gcc (no contraction, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int), ("sort", ctypes.c_int), ("want_v", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("tol", ctypes.c_double),
                ("tthresh", ctypes.c_double), ("block", ctypes.c_int),
                ("max_steps", ctypes.c_long), ("nthreads", ctypes.c_int),
                ("inner_sweeps", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("code", ctypes.c_int), ("rotations", ctypes.c_long),
                ("skips", ctypes.c_long), ("steps", ctypes.c_long), ("r", ctypes.c_int),
                ("inner", ctypes.c_long)]


_lib = None


def load(path: str):
    """Loads an oracle shared library at ``path`` and declares its signatures."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    L.orc_hsvd.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                           ctypes.POINTER(_Params), dp, dp, dp, dp, ip, ctypes.POINTER(_Info)]
    L.orc_hsvd.restype = ctypes.c_int
    L.orc_rotation.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int, dp, dp]
    L.orc_rotation.restype = ctypes.c_int
    L.orc_skip.argtypes = [ctypes.c_double] * 4
    L.orc_skip.restype = ctypes.c_int
    L.orc_conv_code.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_conv_code.restype = ctypes.c_int
    L.orc_pair_params_batch.argtypes = [ctypes.c_long, dp, dp, dp, ip, ctypes.c_double,
                                        ctypes.c_double, ip, dp, dp, ip, ip]
    L.orc_pair_params_batch.restype = None
    L.orc_modmod_init.argtypes = [ctypes.c_int, ip]
    L.orc_modmod_pairs.argtypes = [ctypes.c_int, ip, ip]
    L.orc_modmod_advance.argtypes = [ctypes.c_int, ip]
    L.orc_roundrobin_pairs.argtypes = [ctypes.c_int, ctypes.c_int, ip]
    L.orc_block_step_pairs.argtypes = [ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ip]
    L.orc_block_step_pairs.restype = ctypes.c_int
    L.orc_sort.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip]
    L.orc_bordered_order.argtypes = [ctypes.c_int, ctypes.c_int]
    L.orc_bordered_order.restype = ctypes.c_int
    L.orc_steps_per_sweep.argtypes = [ctypes.c_int, ctypes.c_int]
    L.orc_steps_per_sweep.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load(LIB)
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_tol(n: int) -> float:
    """Skip threshold 1e-15 * n (the workloads' stated tolerance)."""
    return 1e-15 * n


def hsvd(G, p, *, ordering="modmod", sort=True, want_v=True, max_sweeps=100, tol=None,
         tthresh=None, block=0, max_steps=0, nthreads=0, inner_sweeps=0):
    """Run the oracle.  G: (n, n) float64 array (any order).  Returns a dict
    with status, sigma, U, V, lam, perm and the iteration counters."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    assert G.shape == (n, n)
    Gf = np.asfortranarray(G)
    tol = default_tol(n) if tol is None else float(tol)
    tthresh = (np.sqrt(tol) / 2.0) if tthresh is None else float(tthresh)
    prm = _Params(MODMOD if ordering == "modmod" else ROUNDROBIN, int(bool(sort)),
                  int(bool(want_v)), int(max_sweeps), tol, tthresh, int(block),
                  int(max_steps), int(nthreads), int(inner_sweeps))
    sigma = np.zeros(n)
    U = np.zeros((n, n), order="F")
    V = np.zeros((n, n), order="F") if want_v else None
    lam = np.zeros(n)
    perm = np.zeros(n, dtype=np.int32)
    info = _Info()
    st = lib().orc_hsvd(n, int(p), _dp(Gf), n, ctypes.byref(prm), _dp(sigma), _dp(U),
                        _dp(V) if V is not None else None, _dp(lam), _ip(perm),
                        ctypes.byref(info))
    return dict(status=st, sigma=sigma, U=U, V=V, lam=lam, perm=perm, sweeps=info.sweeps,
                code=info.code, rotations=info.rotations, skips=info.skips, steps=info.steps,
                r=info.r, inner=info.inner, tol=tol, tthresh=tthresh)


def rotation(aii, ajj, aij, hyp):
    t = ctypes.c_double()
    c = ctypes.c_double()
    st = lib().orc_rotation(float(aii), float(ajj), float(aij), int(hyp), ctypes.byref(t),
                            ctypes.byref(c))
    return st, t.value, c.value


def skip(aii, ajj, aij, tol):
    return bool(lib().orc_skip(float(aii), float(ajj), float(aij), float(tol)))


def conv_code(code, rotated, t, tthresh):
    return lib().orc_conv_code(int(code), int(rotated), float(t), float(tthresh))


def pair_params_batch(aii, ajj, aij, hyp, tol, tthresh):
    aii = np.ascontiguousarray(aii, dtype=np.float64)
    ajj = np.ascontiguousarray(ajj, dtype=np.float64)
    aij = np.ascontiguousarray(aij, dtype=np.float64)
    hyp = np.ascontiguousarray(hyp, dtype=np.int32)
    m = aii.size
    skip_ = np.zeros(m, np.int32)
    t = np.zeros(m)
    c = np.zeros(m)
    status = np.zeros(m, np.int32)
    code = np.zeros(m, np.int32)
    lib().orc_pair_params_batch(m, _dp(aii), _dp(ajj), _dp(aij), _ip(hyp), float(tol),
                                float(tthresh), _ip(skip_), _dp(t), _dp(c), _ip(status),
                                _ip(code))
    return dict(skip=skip_, t=t, c=c, status=status, code=code)


def modmod_trace(r, steps):
    """(steps, r/2, 2) int array: pairs of the modified modulus strategy."""
    L = lib()
    state = np.zeros(2 * r, np.int32)
    L.orc_modmod_init(r, _ip(state))
    out = np.zeros((steps, r // 2, 2), np.int32)
    buf = np.zeros(r, np.int32)
    for s in range(steps):
        L.orc_modmod_pairs(r, _ip(state), _ip(buf))
        out[s] = buf.reshape(r // 2, 2)
        L.orc_modmod_advance(r, _ip(state))
    return out


def roundrobin_trace(r, steps):
    L = lib()
    out = np.zeros((steps, r // 2, 2), np.int32)
    buf = np.zeros(r, np.int32)
    for s in range(steps):
        L.orc_roundrobin_pairs(r, s % (r - 1), _ip(buf))
        out[s] = buf.reshape(r // 2, 2)
    return out


def block_step_pairs(r, b, outer_pairs, step_in_sweep):
    """All position pairs of one outer step of the block ordering."""
    nb = r // b
    outer = np.ascontiguousarray(np.asarray(outer_pairs, np.int32).reshape(-1))
    assert outer.size == nb
    maxp = (nb // 2) * b * (2 * b - 1)
    buf = np.zeros(2 * maxp, np.int32)
    cnt = lib().orc_block_step_pairs(r, b, _ip(outer), int(step_in_sweep), _ip(buf))
    return buf[: 2 * cnt].reshape(cnt, 2)


def sort_diag(d, rho, p):
    d = np.array(d, dtype=np.float64)
    rho = np.array(rho, dtype=np.int32)
    lib().orc_sort(d.size, int(p), _dp(d), _ip(rho))
    return d, rho


def bordered_order(n, block=0):
    return lib().orc_bordered_order(int(n), int(block))
