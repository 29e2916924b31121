"""ctypes binding of libluqr.so: one Python function per C entry point, same
names, argument marshalling only.  Import fails loudly when the library has
not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LUQR_LIB") or os.path.join(_HERE, "libluqr.so")  # LUQR_LIB: another build of the same ABI

LUQR_ERR_UNSUPPORTED = -900
LUQR_ERR_TOO_LARGE = -901
NOALLOC_SCRATCH_BYTES = 64 << 20
LUQR_ERR_HIP = -1000

CRITERIA = {"max": 0, "sum": 1, "mumps": 2, "random": 3, "forced": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}

EXPORTED = ["luqr_workspace_bytes", "luqr_factor", "luqr_solve", "luqr_solve_refined", "luqr_solve_gmres_ir",
            "luqr_get_decisions", "luqr_get_status", "luqr_get_step_times", "luqr_export_factors", "luqr_destroy",
            "luqr_solve_noalloc", "luqr_alpha_for_growth",
            "luqr_batched_workspace_bytes", "luqr_batched_plan", "luqr_batched_run", "luqr_batched_decision_stride",
            "luqr_batched_destroy", "luqr_batched_autotune"]


class luqr_opts(C.Structure):
    _fields_ = [("nb", C.c_int32), ("criterion", C.c_int32), ("alpha", C.c_double),
                ("precision", C.c_int32), ("nrhs_max", C.c_int32), ("seed", C.c_uint64),
                ("forced", C.POINTER(C.c_int8)), ("nsteps", C.c_int32),
                ("timing", C.c_int32), ("no_lookahead", C.c_int32), ("domain_stride", C.c_int32),
                ("invnorm_estimate", C.c_int32), ("lu_variant", C.c_int32), ("qr_tree", C.c_int32)]


class luqr_status(C.Structure):
    _fields_ = [("info", C.c_int64), ("nonfinite", C.c_int32), ("n_lu", C.c_int32),
                ("ir_iters", C.c_int32), ("ir_converged", C.c_int32), ("ir_eta", C.c_double),
                ("watchdog", C.c_int32), ("reserved", C.c_int32)]


class LuqrError(RuntimeError):
    pass


def check(rc, what):
    if isinstance(rc, int) and rc < 0:
        if rc == LUQR_ERR_UNSUPPORTED:
            raise LuqrError(f"{what}: unsupported option combination")
        if rc == LUQR_ERR_TOO_LARGE:
            raise LuqrError(f"{what}: the problem needs more workspace than the library's buffer holds")
        if rc <= LUQR_ERR_HIP:
            raise LuqrError(f"{what}: HIP error {LUQR_ERR_HIP - rc}")
        raise LuqrError(f"{what}: invalid argument {-rc}")
    return rc


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1401_5522_amd.build` "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    op = C.POINTER(luqr_opts)
    L.luqr_workspace_bytes.restype = i64
    L.luqr_workspace_bytes.argtypes = [i64, op]
    L.luqr_factor.restype = C.c_int
    L.luqr_factor.argtypes = [i64, vp, i64, op, vp, i64, vp, C.POINTER(vp)]
    L.luqr_solve.restype = C.c_int
    L.luqr_solve.argtypes = [vp, i64, vp, i64, vp]
    L.luqr_solve_refined.restype = C.c_int
    L.luqr_solve_refined.argtypes = [vp, vp, i64, i64, vp, i64, vp, i64, i32, vp]
    L.luqr_solve_gmres_ir.restype = C.c_int
    L.luqr_solve_gmres_ir.argtypes = [vp, vp, i64, vp, vp, i32, i32, C.POINTER(C.c_int32), vp]
    L.luqr_alpha_for_growth.restype = C.c_double
    L.luqr_alpha_for_growth.argtypes = [i64, i32, i32, C.c_double]
    L.luqr_get_decisions.restype = C.c_int
    L.luqr_get_decisions.argtypes = [vp, vp, vp, vp, vp, i64]
    L.luqr_get_status.restype = C.c_int
    L.luqr_get_status.argtypes = [vp, C.POINTER(luqr_status)]
    L.luqr_get_step_times.restype = C.c_int
    L.luqr_get_step_times.argtypes = [vp, vp, i64]
    L.luqr_export_factors.restype = C.c_int
    L.luqr_export_factors.argtypes = [vp, vp, i64, vp, vp]
    L.luqr_destroy.restype = None
    L.luqr_destroy.argtypes = [vp]
    L.luqr_solve_noalloc.restype = C.c_int
    L.luqr_solve_noalloc.argtypes = [i64, vp, i64, op, i64, vp, i64, vp, i64, i32, C.POINTER(luqr_status), vp]
    L.luqr_batched_workspace_bytes.restype = i64
    L.luqr_batched_workspace_bytes.argtypes = [i64, vp, vp, op]
    L.luqr_batched_plan.restype = C.c_int
    L.luqr_batched_plan.argtypes = [i64, vp, vp, vp, vp, vp, op, i32, vp, i64, C.POINTER(vp)]
    L.luqr_batched_run.restype = C.c_int
    L.luqr_batched_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.luqr_batched_decision_stride.restype = C.c_int
    L.luqr_batched_decision_stride.argtypes = [vp]
    L.luqr_batched_destroy.restype = None
    L.luqr_batched_destroy.argtypes = [vp]
    L.luqr_batched_autotune.restype = C.c_int
    L.luqr_batched_autotune.argtypes = [i64, vp, vp, vp, vp, op, i32, vp, vp, vp, i32, vp, i64, vp, vp, vp]
    _lib = L
    return L


def make_opts(nb, criterion="max", alpha=1.0, precision="fp64", nrhs_max=1, seed=0, forced=None,
              nsteps=-1, timing=False, lookahead=True, domain=0, estimate=False, variant=1, tree=0):
    o = luqr_opts()
    o.nb = int(nb)
    o.criterion = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    o.alpha = float(alpha)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.nrhs_max = int(nrhs_max)
    o.seed = int(seed)
    keep = None
    if forced is not None:
        keep = (C.c_int8 * len(forced))(*[int(v) for v in forced])
        o.forced = C.cast(keep, C.POINTER(C.c_int8))
    o.nsteps = int(nsteps)
    o.timing = 1 if timing else 0
    o.no_lookahead = 0 if lookahead else 1
    o.domain_stride = int(domain)
    o.invnorm_estimate = 1 if estimate else 0
    o.lu_variant = int(variant)
    o.qr_tree = int(tree)
    return o, keep


# ---- thin wrappers, same names as the C ABI ---------------------------------

def luqr_workspace_bytes(N, opts):
    return check(lib().luqr_workspace_bytes(N, C.byref(opts)), "luqr_workspace_bytes")


def luqr_factor(N, dA, lda, opts, dWork, work_bytes, stream):
    h = C.c_void_p()
    check(lib().luqr_factor(N, dA, lda, C.byref(opts), dWork, work_bytes, stream, C.byref(h)), "luqr_factor")
    return h


def luqr_solve(h, nrhs, dB, ldb, stream):
    return check(lib().luqr_solve(h, nrhs, dB, ldb, stream), "luqr_solve")


def luqr_solve_refined(h, dA, lda, nrhs, dB, ldb, dX, ldx, max_iter, stream):
    return check(lib().luqr_solve_refined(h, dA, lda, nrhs, dB, ldb, dX, ldx, max_iter, stream),
                 "luqr_solve_refined")


def luqr_solve_gmres_ir(h, dA, lda, db, dx, max_outer, max_inner, stream):
    inner = C.c_int32(0)
    check(lib().luqr_solve_gmres_ir(h, dA, lda, db, dx, max_outer, max_inner, C.byref(inner), stream),
          "luqr_solve_gmres_ir")
    return inner.value


def luqr_alpha_for_growth(N, nb, criterion, growth):
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    a = lib().luqr_alpha_for_growth(int(N), int(nb), crit, float(growth))
    if a < 0:
        raise LuqrError(f"luqr_alpha_for_growth: invalid argument {int(-a)}")
    return a


def luqr_get_decisions(h, dec, s, m, margin, n):
    return check(lib().luqr_get_decisions(h, dec, s, m, margin, n), "luqr_get_decisions")


def luqr_get_status(h):
    st = luqr_status()
    check(lib().luqr_get_status(h, C.byref(st)), "luqr_get_status")
    return st


NPHASE = 5  # LUQR_NPHASE: panel, LU apply, LU update, QR step, R^-1


def luqr_get_step_times(h, t, n):
    return check(lib().luqr_get_step_times(h, t, n), "luqr_get_step_times")


def luqr_export_factors(h, dF, ldf, ipiv, stream):
    return check(lib().luqr_export_factors(h, dF, ldf, ipiv, stream), "luqr_export_factors")


def luqr_destroy(h):
    lib().luqr_destroy(h)


def luqr_solve_noalloc(N, dA, lda, opts, nrhs, dB, ldb, dX, ldx, max_iter, stream):
    st = luqr_status()
    check(lib().luqr_solve_noalloc(N, dA, lda, C.byref(opts), nrhs, dB, ldb, dX, ldx, max_iter, C.byref(st),
                                   stream), "luqr_solve_noalloc")
    return st


def luqr_batched_workspace_bytes(batch, N, nb, opts):
    return check(lib().luqr_batched_workspace_bytes(batch, N, nb, C.byref(opts)), "luqr_batched_workspace_bytes")


def luqr_batched_plan(batch, N, nb, lda, ldb, ldx, opts, max_iter, dWork, work_bytes):
    h = C.c_void_p()
    check(lib().luqr_batched_plan(batch, N, nb, lda, ldb, ldx, C.byref(opts), max_iter, dWork, work_bytes,
                                  C.byref(h)), "luqr_batched_plan")
    return h


def luqr_batched_run(plan, dA, dB, dX, dDec, dEta, dIters, stream):
    return check(lib().luqr_batched_run(plan, dA, dB, dX, dDec, dEta, dIters, stream), "luqr_batched_run")


def luqr_batched_decision_stride(plan):
    return check(lib().luqr_batched_decision_stride(plan), "luqr_batched_decision_stride")


def luqr_batched_destroy(plan):
    lib().luqr_batched_destroy(plan)


def luqr_batched_autotune(batch, N, lda, ldb, ldx, opts, max_iter, dA, dB, dX, sample, dWork, work_bytes, stream,
                          nb_out, ms_out):
    return check(lib().luqr_batched_autotune(batch, N, lda, ldb, ldx, C.byref(opts), max_iter, dA, dB, dX, sample,
                                             dWork, work_bytes, stream, nb_out, ms_out), "luqr_batched_autotune")
