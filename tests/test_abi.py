"""The C-ABI library loads and exports every entry point include/luqr.h
declares; argument validation that needs no GPU returns the documented codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "luqr.h")).read()
    return sorted(set(re.findall(r"\b(luqr_[a-z_]+)\s*\(", txt)))


def test_header_lists_the_binding_names():
    from paper_1401_5522_amd import _lib
    assert header_symbols() == sorted(_lib.EXPORTED)


def test_library_exports_every_symbol():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    for name in header_symbols():
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    from paper_1401_5522_amd import _lib
    assert C.sizeof(_lib.luqr_opts) == 72
    assert _lib.luqr_opts.invnorm_estimate.offset == 56
    assert _lib.luqr_opts.lu_variant.offset == 60
    assert _lib.luqr_opts.qr_tree.offset == 64
    assert _lib.luqr_opts.forced.offset == 32
    assert C.sizeof(_lib.luqr_status) == 40
    assert _lib.luqr_status.ir_eta.offset == 24


def test_workspace_bytes_validation_without_gpu():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    o, _ = _lib.make_opts(128)
    assert L.luqr_workspace_bytes(1024, C.byref(o)) > 1024 * 1024 * 8
    assert L.luqr_workspace_bytes(0, C.byref(o)) == -1
    o.alpha = -1.0
    assert L.luqr_workspace_bytes(1024, C.byref(o)) == -2
    o, _ = _lib.make_opts(100)                       # tile size without kernels
    assert L.luqr_workspace_bytes(1024, C.byref(o)) == _lib.LUQR_ERR_UNSUPPORTED
    o, _ = _lib.make_opts(512, precision="fp64")     # FP64 at nb=512 is not built
    assert L.luqr_workspace_bytes(4096, C.byref(o)) == _lib.LUQR_ERR_UNSUPPORTED
    o, _ = _lib.make_opts(64, criterion="forced")    # FORCED without a sequence
    assert L.luqr_workspace_bytes(256, C.byref(o)) == -2
    o, _ = _lib.make_opts(64, alpha=float("nan"))
    assert L.luqr_workspace_bytes(256, C.byref(o)) == -2


def test_factor_rejects_bad_arguments_before_any_gpu_call():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    o, _ = _lib.make_opts(64)
    h = C.c_void_p()
    assert L.luqr_factor(0, C.c_void_p(16), 1, C.byref(o), C.c_void_p(256), 1 << 30, None, C.byref(h)) == -1
    assert L.luqr_factor(64, None, 64, C.byref(o), C.c_void_p(256), 1 << 30, None, C.byref(h)) == -2
    assert L.luqr_factor(64, C.c_void_p(16), 10, C.byref(o), C.c_void_p(256), 1 << 30, None, C.byref(h)) == -3
    assert L.luqr_factor(64, C.c_void_p(16), 64, C.byref(o), C.c_void_p(100), 1 << 30, None, C.byref(h)) == -5
    assert L.luqr_factor(64, C.c_void_p(16), 64, C.byref(o), C.c_void_p(256), 10, None, C.byref(h)) == -6
    assert L.luqr_solve(None, 1, None, 1, None) == -1


def test_domain_stride_validation_without_gpu():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    o, _ = _lib.make_opts(128, domain=2)                 # n = 8: 1 + 7/2 = 4 tiles, 512 rows
    assert L.luqr_workspace_bytes(1024, C.byref(o)) > 0
    o, _ = _lib.make_opts(128, domain=1)                 # 8 tiles of 128 rows: more than 512
    assert L.luqr_workspace_bytes(1024, C.byref(o)) == _lib.LUQR_ERR_UNSUPPORTED
    o, _ = _lib.make_opts(128, domain=-1)
    assert L.luqr_workspace_bytes(1024, C.byref(o)) == -2


def test_lu_variant_validation_without_gpu():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    for v in (0, 1, 2):
        o, _ = _lib.make_opts(64, variant=v)
        assert L.luqr_workspace_bytes(256, C.byref(o)) > 0
    o, _ = _lib.make_opts(64, variant=3)
    assert L.luqr_workspace_bytes(256, C.byref(o)) == -2
    o, _ = _lib.make_opts(64, variant=-1)
    assert L.luqr_workspace_bytes(256, C.byref(o)) == -2
    # A2 has no GEPP pivots (MUMPS), no stacked domain and no unit-lower L^-1 (estimate)
    for kw in (dict(criterion="mumps"), dict(domain=1), dict(estimate=True)):
        o, _ = _lib.make_opts(64, variant=2, **kw)
        assert L.luqr_workspace_bytes(256, C.byref(o)) == _lib.LUQR_ERR_UNSUPPORTED, kw
    o, _ = _lib.make_opts(64, precision="fp32", variant=2)  # batched: FP32 and A1 only, checked before any GPU call
    plan = C.c_void_p()
    Ns = np.array([64], np.int64)
    ld = np.array([64], np.int64)
    rc = L.luqr_batched_plan(1, Ns.ctypes.data, None, ld.ctypes.data, ld.ctypes.data, ld.ctypes.data, C.byref(o),
                             4, C.c_void_p(256), 1 << 30, C.byref(plan))
    assert rc == _lib.LUQR_ERR_UNSUPPORTED


def test_qr_tree_validation_without_gpu():
    from paper_1401_5522_amd import _lib
    L = _lib.lib()
    o0, _ = _lib.make_opts(64)
    o1, _ = _lib.make_opts(64, tree=2)
    b0 = L.luqr_workspace_bytes(1024, C.byref(o0))
    b1 = L.luqr_workspace_bytes(1024, C.byref(o1))
    n = 1024 // 64
    # one more T factor per panel tile (in place of a 256-byte placeholder)
    assert b1 - b0 == n * (n + 1) // 2 * 64 * 64 * 8 - 256
    o, _ = _lib.make_opts(64, tree=-1)
    assert L.luqr_workspace_bytes(1024, C.byref(o)) == -2
    o, _ = _lib.make_opts(64, precision="fp32", tree=2)
    plan = C.c_void_p()
    Ns = np.array([64], np.int64)
    ld = np.array([64], np.int64)
    rc = L.luqr_batched_plan(1, Ns.ctypes.data, None, ld.ctypes.data, ld.ctypes.data, ld.ctypes.data, C.byref(o),
                             4, C.c_void_p(256), 1 << 30, C.byref(plan))
    assert rc == _lib.LUQR_ERR_UNSUPPORTED
