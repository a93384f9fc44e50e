"""ctypes binding of libhsvd.so (include/hsvd.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Matrices are passed
as torch tensors holding the mathematical matrix; a column-major view
(``X.t()`` of a contiguous ``X``) is passed through without a copy, anything
else is copied to column-major storage first.

Importing this module does not touch the GPU.  Loading the library fails
loudly when it has not been built (``python -m paper_1008_1371_amd.build``).
"""
from __future__ import annotations

import collections.abc
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsvd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hsvd.h")

OK, E_INVAL, E_NOCONV, E_RANK, E_NOMEM, E_DEVICE, E_SIZE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOCONV", -3: "E_RANK", -4: "E_NOMEM",
                -5: "E_DEVICE", -6: "E_SIZE"}
NOALLOC_BYTES = 64 << 20  # HSVD_NOALLOC_BYTES
FP64, MIXED = 0, 1
AUTO, PAIRWISE, BLOCK = 0, 1, 2
MODMOD, ROUNDROBIN = 0, 1


class hsvd_params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("algo", ctypes.c_int), ("ordering", ctypes.c_int),
                ("block", ctypes.c_int), ("sort", ctypes.c_int), ("want_v", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("tol", ctypes.c_double),
                ("t_thresh", ctypes.c_double), ("graph", ctypes.c_int),
                ("inner_sweeps", ctypes.c_int), ("reorth_accept", ctypes.c_double),
                ("batch_mode", ctypes.c_int), ("persistent", ctypes.c_int)]


NKERNELS = 8
(K_PAIR_STEP, K_BLOCK_GRAM, K_BLOCK_INNER, K_BLOCK_UPDATE, K_BLOCK_GRAM32, K_BLOCK_INNER32,
 K_BLOCK_UPDATE32, K_REORTH) = range(NKERNELS)
KERNEL_NAMES = ["pair_step_kernel", "block_gram_kernel<double>", "block_inner_kernel<double>",
                "block_update_kernel<double>", "block_gram_kernel<float>",
                "block_inner_kernel<float>", "block_update_kernel<float>", "gemm_f64_kernel (reorth)"]


class hsvd_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sweeps", ctypes.c_int), ("code", ctypes.c_int),
                ("r", ctypes.c_int), ("block", ctypes.c_int), ("ldg", ctypes.c_int),
                ("sweeps_fp32", ctypes.c_int), ("reorth_iters", ctypes.c_int),
                ("max_t_last", ctypes.c_double), ("reorth_resid", ctypes.c_double),
                ("fp64_restart", ctypes.c_int), ("pad_", ctypes.c_int),
                ("rotations", ctypes.c_longlong), ("skips", ctypes.c_longlong),
                ("steps", ctypes.c_longlong), ("active_pairs", ctypes.c_longlong),
                ("ms_total", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * NKERNELS),
                ("kernel_launches", ctypes.c_longlong * NKERNELS),
                ("kernel_bytes", ctypes.c_double * NKERNELS),
                ("kernel_flops", ctypes.c_double * NKERNELS),
                ("kernel_timed", ctypes.c_longlong * NKERNELS)]

    def as_dict(self):
        out = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            out[k] = list(v) if hasattr(v, "__len__") else v
        return out


class InfoList(collections.abc.Sequence):
    """The per-problem hsvd_info of a batched solve as a sequence of dicts,
    each converted when it is accessed (converting 10^4 of them up front
    takes longer than a small batch's solve)."""

    def __init__(self, arr, n):
        self._a = arr
        self._n = n

    def __len__(self):
        return self._n

    def __getitem__(self, k):
        if isinstance(k, slice):
            return [self._a[i].as_dict() for i in range(*k.indices(self._n))]
        if k < 0:
            k += self._n
        if not 0 <= k < self._n:
            raise IndexError(k)
        return self._a[k].as_dict()


_lib = None


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/hsvd.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return re.findall(r"\b(hsvd_\w+)\s*\(", txt)


def lib():
    """Loads libhsvd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1008_1371_amd.build` (there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.hsvd_init.argtypes = [ctypes.POINTER(vp), ip, vp]
    L.hsvd_destroy.argtypes = [vp]
    L.hsvd_default_params.argtypes = [ctypes.POINTER(hsvd_params)]
    L.hsvd_default_params.restype = None
    L.hsvd_solve.argtypes = [vp, vp, ip, vp, ip, ip, ctypes.POINTER(hsvd_params), vp, vp, ip, vp, ip,
                             vp, vp, ctypes.POINTER(hsvd_info)]
    L.hsvd_pair_params.argtypes = [vp, ctypes.c_longlong, vp, vp, vp, vp, dp, dp, vp, vp, vp, vp,
                                   vp]
    L.hsvd_block_pair_params.argtypes = L.hsvd_pair_params.argtypes
    L.hsvd_autotune.argtypes = [vp, ip, ctypes.POINTER(ip), ctypes.POINTER(ip)]
    L.hsvd_pivot_trace.argtypes = [vp, ip, ip, ip, vp]
    L.hsvd_sort_diag.argtypes = [vp, ip, ip, vp, vp]
    L.hsvd_block_trace.argtypes = [vp, ip, ip, ip, ip, vp]
    L.hsvd_solve_noalloc.argtypes = [vp, vp, ip, ip, ip, ctypes.POINTER(hsvd_params), vp, vp, ip, vp, ip,
                                     vp, vp, ctypes.POINTER(hsvd_info)]
    L.hsvd_solve_batched.argtypes = [vp, ip, vp, vp, vp, vp, vp, ctypes.POINTER(hsvd_params), vp, vp,
                                     vp, vp, vp]
    L.hsvd_autotune_batched.argtypes = [vp, ip, vp, vp, ctypes.POINTER(ip), vp]
    L.hsvd_batched_schedule.argtypes = [vp, ip, ctypes.POINTER(ip)]
    L.hsvd_version.restype = ctypes.c_char_p
    for name in ("hsvd_init", "hsvd_destroy", "hsvd_solve", "hsvd_solve_noalloc", "hsvd_autotune",
                 "hsvd_pair_params",
                 "hsvd_block_pair_params",
                 "hsvd_pivot_trace", "hsvd_sort_diag", "hsvd_block_trace", "hsvd_solve_batched",
                 "hsvd_autotune_batched", "hsvd_batched_schedule"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class HsvdError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


def _check(st, what):
    if st != OK:
        raise HsvdError(st, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _colmajor(G):
    """Returns (tensor, ld) with column-major storage of the matrix G."""
    import torch  # noqa: F401  (device memory and streams only)
    n0, n1 = G.shape
    if G.stride(0) == 1 and G.stride(1) >= max(1, n0):
        return G, G.stride(1)
    Gc = G.t().contiguous().t()
    return Gc, n0


def _new_colmajor(n, device, dtype):
    import torch
    return torch.empty((n, n), dtype=dtype, device=device).t()


class Context:
    """An hsvd_ctx bound to a device and a stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(L.hsvd_init(ctypes.byref(h), int(device), ctypes.c_void_p(stream)), "hsvd_init")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().hsvd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def hsvd_init(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


def hsvd_destroy(ctx: Context) -> None:
    ctx.close()


def hsvd_default_params(**overrides) -> hsvd_params:
    prm = hsvd_params()
    lib().hsvd_default_params(ctypes.byref(prm))
    for k, v in overrides.items():
        setattr(prm, k, v)
    return prm


def hsvd_solve(ctx: Context, G, p: int | None = None, params: hsvd_params | None = None, *, jsig=None,
               want_u=True, want_v=None, want_lambda=True, want_perm=True, out=None, check=True, noalloc=False):
    """Solves G = U Sigma V^T, V^T J V = J.

    G: square float64 CUDA tensor.  J = diag(I_p, -I_{n-p}), or, with jsig (an
    int8 CUDA tensor of +-1 entries, one per column of G, in any order), J =
    diag(jsig) and p its number of +1 entries.  Returns a dict with sigma, U,
    V, lambda, perm (tensors or None), status and info (a dict).  ``out`` may
    hold preallocated output tensors with the same keys."""
    import torch
    L = lib()
    n = G.shape[0]
    assert G.shape == (n, n) and G.dtype == torch.float64 and G.is_cuda
    if jsig is not None:
        assert jsig.dtype == torch.int8 and jsig.numel() == n and jsig.is_cuda
        jsig = jsig.contiguous()
        if p is None:
            p = int((jsig == 1).sum().item())
    assert p is not None
    prm = params if params is not None else hsvd_default_params()
    if want_v is None:
        want_v = bool(prm.want_v)
    Gc, lda = _colmajor(G)
    out = dict(out or {})
    dev = G.device
    sigma = out.get("sigma")
    if sigma is None:
        sigma = torch.empty(n, dtype=torch.float64, device=dev)
    U = out.get("U") if want_u else None
    if want_u and U is None:
        U = _new_colmajor(n, dev, torch.float64)
    V = out.get("V") if want_v else None
    if want_v and V is None:
        V = _new_colmajor(n, dev, torch.float64)
    lam = out.get("lambda") if want_lambda else None
    if want_lambda and lam is None:
        lam = torch.empty(n, dtype=torch.float64, device=dev)
    perm = out.get("perm") if want_perm else None
    if want_perm and perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    info = hsvd_info()
    ldu = U.stride(1) if U is not None else n
    ldv = V.stride(1) if V is not None else n
    if noalloc:
        assert jsig is None, "hsvd_solve_noalloc takes J = diag(I_p, -I_{n-p})"
        name = "hsvd_solve_noalloc"
        st = L.hsvd_solve_noalloc(ctx.handle, _ptr(Gc), lda, n, int(p), ctypes.byref(prm), _ptr(sigma), _ptr(U),
                                  ldu, _ptr(V), ldv, _ptr(lam), _ptr(perm), ctypes.byref(info))
    else:
        name = "hsvd_solve"
        st = L.hsvd_solve(ctx.handle, _ptr(Gc), lda, _ptr(jsig), n, int(p), ctypes.byref(prm), _ptr(sigma),
                          _ptr(U), ldu, _ptr(V), ldv, _ptr(lam), _ptr(perm), ctypes.byref(info))
    if check and st not in (OK,):
        raise HsvdError(st, name)
    return dict(status=st, sigma=sigma, U=U, V=V, lam=lam, perm=perm, info=info.as_dict())


def hsvd_solve_noalloc(ctx: Context, G, p: int, params: hsvd_params | None = None, **kw):
    """hsvd_solve through the entry point that allocates no device memory
    (the library's fixed scratch array; J = diag(I_p, -I_{n-p})).  Output
    tensors are allocated here unless passed in ``out``."""
    return hsvd_solve(ctx, G, p, params, noalloc=True, **kw)


def hsvd_autotune(ctx: Context, n: int):
    """Tunes the path and the Gram split for n's size bucket; returns (algo, wg)."""
    a = ctypes.c_int()
    w = ctypes.c_int()
    _check(lib().hsvd_autotune(ctx.handle, int(n), ctypes.byref(a), ctypes.byref(w)), "hsvd_autotune")
    return a.value, w.value


def hsvd_batched_schedule(ctx: Context, precision: int) -> int:
    """The sweep schedule batch_mode 2 takes for `precision`: 0 persistent,
    1 grouped, -1 not tuned."""
    m = ctypes.c_int()
    _check(lib().hsvd_batched_schedule(ctx.handle, int(precision), ctypes.byref(m)), "hsvd_batched_schedule")
    return m.value


def hsvd_autotune_batched(ctx: Context, ns, ps):
    """Times the persistent batched kernel's widths (256 / 512 / 1024 threads
    per problem) on a sample of the given orders and keeps the fastest for
    their size bucket, then the two sweep schedules per precision; returns
    (threads, {threads: ms})."""
    import numpy as np
    n_a = np.ascontiguousarray(ns, dtype=np.int32)
    p_a = np.ascontiguousarray(ps, dtype=np.int32)
    best = ctypes.c_int()
    ms = (ctypes.c_float * 3)()
    _check(lib().hsvd_autotune_batched(ctx.handle, int(n_a.size), n_a.ctypes.data_as(ctypes.c_void_p),
                                       p_a.ctypes.data_as(ctypes.c_void_p), ctypes.byref(best), ms),
           "hsvd_autotune_batched")
    return best.value, {256: ms[0], 512: ms[1], 1024: ms[2]}


def hsvd_solve_batched(ctx: Context, ns, ps, G_packed, offs, voffs, params: hsvd_params | None = None,
                       *, want_u=True, want_v=None, want_lambda=True, out=None, check=True):
    """Solves many independent problems in one call.

    ns, ps, offs, voffs: integer sequences (order, +1 signs, element offset of
    each column-major G_k in G_packed, offset of sigma_k), passed to the
    library as device arrays.  G_packed: float64 CUDA tensor with all inputs.
    Returns a dict with the packed outputs (sigma, U, V, lam: tensors or
    None), the per-problem infos (a sequence of dicts, each converted when
    accessed) and, for convenience, their statuses and FP64 sweep counts as
    NumPy arrays."""
    import numpy as np
    import torch
    L = lib()
    batch = len(ns)
    prm = params if params is not None else hsvd_default_params()
    if want_v is None:
        want_v = bool(prm.want_v)
    dev = G_packed.device
    n_a = np.ascontiguousarray(ns, dtype=np.int32)
    v_a = np.ascontiguousarray(voffs, dtype=np.int64)
    n_d = torch.from_numpy(n_a).to(dev)
    p_d = torch.from_numpy(np.ascontiguousarray(ps, dtype=np.int32)).to(dev)
    o_d = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.int64)).to(dev)
    v_d = torch.from_numpy(v_a).to(dev)
    tot_v = int((v_a + n_a).max()) if batch else 0
    out = dict(out or {})
    sigma = out.get("sigma")
    if sigma is None:
        sigma = torch.empty(tot_v, dtype=torch.float64, device=dev)
    U = out.get("U") if want_u else None
    if want_u and U is None:
        U = torch.empty_like(G_packed)
    V = out.get("V") if want_v else None
    if want_v and V is None:
        V = torch.empty_like(G_packed)
    lam = out.get("lambda") if want_lambda else None
    if want_lambda and lam is None:
        lam = torch.empty(tot_v, dtype=torch.float64, device=dev)
    infos = (hsvd_info * max(batch, 1))()
    st = L.hsvd_solve_batched(ctx.handle, batch, _ptr(n_d), _ptr(p_d), _ptr(o_d), _ptr(v_d), _ptr(G_packed),
                              ctypes.byref(prm), _ptr(sigma), _ptr(U), _ptr(V), _ptr(lam), infos)
    if check and st != OK:
        raise HsvdError(st, "hsvd_solve_batched")
    rec = np.ctypeslib.as_array(infos)[:batch]
    status = rec["status"].astype(np.int32)
    sweeps = rec["sweeps"].astype(np.int32)
    return dict(status=st, sigma=sigma, U=U, V=V, lam=lam, infos=InfoList(infos, batch), statuses=status,
                sweeps=sweeps)


def hsvd_pair_params(ctx: Context, aii, ajj, aij, hyp, tol: float, t_thresh: float, block=False):
    import torch
    m = aii.numel()
    dev = aii.device
    skip = torch.empty(m, dtype=torch.int32, device=dev)
    status = torch.empty(m, dtype=torch.int32, device=dev)
    code = torch.empty(m, dtype=torch.int32, device=dev)
    t = torch.empty(m, dtype=torch.float64, device=dev)
    c = torch.empty(m, dtype=torch.float64, device=dev)
    fn = lib().hsvd_block_pair_params if block else lib().hsvd_pair_params
    _check(fn(ctx.handle, m, _ptr(aii), _ptr(ajj), _ptr(aij), _ptr(hyp), float(tol), float(t_thresh),
              _ptr(skip), _ptr(t), _ptr(c), _ptr(status), _ptr(code)), "hsvd_pair_params")
    return dict(skip=skip, t=t, c=c, status=status, code=code)


def hsvd_pivot_trace(ctx: Context, ordering: int, r: int, steps: int):
    import torch
    pairs = torch.empty((steps, r // 2, 2), dtype=torch.int32, device=f"cuda:{ctx.device}")
    _check(lib().hsvd_pivot_trace(ctx.handle, int(ordering), int(r), int(steps), _ptr(pairs)),
           "hsvd_pivot_trace")
    return pairs


def hsvd_sort_diag(ctx: Context, d, rho, p: int):
    _check(lib().hsvd_sort_diag(ctx.handle, d.numel(), int(p), _ptr(d), _ptr(rho)),
           "hsvd_sort_diag")
    return d, rho


def hsvd_version() -> str:
    return lib().hsvd_version().decode()
