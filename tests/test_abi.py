"""The C ABI library loads and exports every function include/hsvd.h declares.
No compute calls (CPU only)."""
import ctypes
import os

import pytest

from paper_1008_1371_amd import hsvd as H


def _lib_or_skip():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhsvd.so not built (run __graft_entry__.build())")
    return H.lib()


def test_header_declares_the_entry_points():
    names = H.header_functions()
    for required in ("hsvd_init", "hsvd_destroy", "hsvd_default_params", "hsvd_solve",
                     "hsvd_pair_params", "hsvd_block_pair_params", "hsvd_pivot_trace",
                     "hsvd_sort_diag", "hsvd_block_trace", "hsvd_solve_batched", "hsvd_version",
                     "hsvd_solve_noalloc"):
        assert required in names


def test_every_declared_symbol_is_exported():
    L = _lib_or_skip()
    missing = [nm for nm in H.header_functions() if not hasattr(L, nm)]
    assert not missing, missing


def test_defaults_and_argument_checks_without_gpu():
    L = _lib_or_skip()
    prm = H.hsvd_default_params()
    assert (prm.precision, prm.algo, prm.ordering, prm.sort, prm.want_v, prm.max_sweeps,
            prm.graph, prm.inner_sweeps, prm.reorth_accept, prm.batch_mode, prm.persistent) == \
        (H.FP64, H.AUTO, H.MODMOD, 1, 1, 100, 1, 0, 0.0, 2, 0)
    assert H.hsvd_version().startswith("hsvd-gfx950")
    # argument errors are reported before any device call
    assert L.hsvd_init(None, 0, None) == H.E_INVAL
    assert L.hsvd_destroy(None) == H.E_INVAL
    info = H.hsvd_info()
    assert L.hsvd_solve(None, None, 1, None, 1, 0, None, None, None, 1, None, 1, None, None,
                        ctypes.byref(info)) == H.E_INVAL
    assert L.hsvd_solve_noalloc(None, None, 1, 1, 0, None, None, None, 1, None, 1, None, None,
                                ctypes.byref(info)) == H.E_INVAL
    assert L.hsvd_pivot_trace(None, 0, 4, 1, None) == H.E_INVAL
    assert L.hsvd_block_trace(None, 0, 64, 32, 1, None) == H.E_INVAL
    assert L.hsvd_solve_batched(None, 1, None, None, None, None, None, None, None, None, None, None,
                                ctypes.byref(info)) == H.E_INVAL
    assert L.hsvd_block_pair_params(None, 1, None, None, None, None, 0.0, 0.0, None, None, None,
                                    None, None) == H.E_INVAL


def test_struct_layouts_match_header():
    # field order and count of the ctypes mirrors against the header text
    txt = open(H.HEADER).read()
    for struct, cls in (("hsvd_params", H.hsvd_params), ("hsvd_info", H.hsvd_info)):
        body = txt.split("typedef struct {", 1)[1] if struct == "hsvd_params" else \
            txt.split("typedef struct {", 2)[2]
        body = body.split("} " + struct + ";")[0]
        import re
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"\b(\w+)\s*(?:\[\w+\])?\s*;", body)
        assert fields == [f for f, _ in cls._fields_], (struct, fields)
