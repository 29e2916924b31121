"""ctypes binding of the plain FP64 CPU oracle (``luqr_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product package.  It shares no
code with the HIP implementation.

Every function takes and returns numpy arrays in column-major (Fortran) order.
See the header comment of ``luqr_oracle.c`` for the storage conventions and the
paper passages each routine follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "luqr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CRITERIA = {"max": 0, "sum": 1, "mumps": 2, "random": 3, "forced": 4}

DG_INFO, DG_NONFINITE, DG_GROWTH_TILE, DG_GROWTH_ELEM, DG_MAXINEQ, DG_SUMINEQ, DG_TRUEFLOPS, DG_NLU = range(8)
DG_COUNT = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP across independent tiles).

    ``-ffp-contract=off`` keeps every multiply and add rounded as written.
    """
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        i64, i32, f64 = C.c_int64, C.c_int32, C.c_double
        dp, ip, bp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int8)
        L.oracle_factor.restype = C.c_int
        L.oracle_factor.argtypes = [i64, dp, i64, i64, i32, f64, C.c_uint64, bp, i32, i64,
                                    dp, i64, i64, ip, dp, bp, dp, dp, dp, dp]
        L.oracle_factor_domain.restype = C.c_int
        L.oracle_factor_domain.argtypes = [i64, dp, i64, i64, i32, f64, C.c_uint64, bp, i32, i64,
                                           dp, i64, i64, ip, dp, bp, dp, dp, dp, dp, i32]
        L.oracle_factor_ex.restype = C.c_int
        L.oracle_factor_ex.argtypes = [i64, dp, i64, i64, i32, f64, C.c_uint64, bp, i32, i64,
                                       dp, i64, i64, ip, dp, bp, dp, dp, dp, dp, i32, i32, i32]
        L.oracle_factor_t.restype = C.c_int
        L.oracle_factor_t.argtypes = [i64, dp, i64, i64, i32, f64, C.c_uint64, bp, i32, i64,
                                      dp, i64, i64, ip, dp, bp, dp, dp, dp, dp, i32, i32, i32, i32, dp]
        L.oracle_solve_t.restype = None
        L.oracle_solve_t.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32, i32, i32, dp]
        L.oracle_forward_t.restype = None
        L.oracle_forward_t.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32, i32, i32, dp]
        L.oracle_ttqrt.restype = None
        L.oracle_ttqrt.argtypes = [i64, dp, i64, dp, i64, dp, i64]
        L.oracle_ttmqr.restype = None
        L.oracle_ttmqr.argtypes = [i64, dp, i64, dp, i64, i64, dp, i64, dp, i64]
        L.oracle_inv_norm1_qr.restype = f64
        L.oracle_inv_norm1_qr.argtypes = [i64, dp, i64, dp, i64]
        L.oracle_solve_v.restype = None
        L.oracle_solve_v.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32, i32]
        L.oracle_forward_v.restype = None
        L.oracle_forward_v.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32, i32]
        L.oracle_inv_norm1_est.restype = f64
        L.oracle_inv_norm1_est.argtypes = [i64, dp, i64]
        L.oracle_solve.restype = None
        L.oracle_solve.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64]
        L.oracle_solve_domain.restype = None
        L.oracle_solve_domain.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32]
        L.oracle_forward.restype = None
        L.oracle_forward.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64]
        L.oracle_forward_domain.restype = None
        L.oracle_forward_domain.argtypes = [i64, dp, i64, i64, ip, dp, bp, dp, i64, i64, i32]
        L.oracle_backward.restype = None
        L.oracle_backward.argtypes = [i64, dp, i64, i64, dp, i64, i64]
        L.oracle_gepp.restype = i64
        L.oracle_gepp.argtypes = [i64, dp, i64, ip]
        L.oracle_inv_norm1.restype = f64
        L.oracle_inv_norm1.argtypes = [i64, dp, i64, ip]
        L.oracle_tile_norm1.restype = f64
        L.oracle_tile_norm1.argtypes = [dp, i64, i64, i64]
        L.oracle_geqrt.restype = None
        L.oracle_geqrt.argtypes = [i64, dp, i64, dp, i64]
        L.oracle_unmqr.restype = None
        L.oracle_unmqr.argtypes = [i64, dp, i64, dp, i64, i64, dp, i64]
        L.oracle_tsqrt.restype = None
        L.oracle_tsqrt.argtypes = [i64, dp, i64, i64, dp, i64, dp, i64]
        L.oracle_tsmqr.restype = None
        L.oracle_tsmqr.argtypes = [i64, i64, dp, i64, dp, i64, i64, dp, i64, dp, i64]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_uniform.restype = f64
        L.oracle_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_true_flops.restype = f64
        L.oracle_true_flops.argtypes = [i64, i64, bp]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _b(a):
    return a.ctypes.data_as(C.POINTER(C.c_int8)) if a is not None else None


def _fortran(a, dtype=np.float64):
    return np.array(a, dtype=dtype, order="F", copy=True)


@dataclass
class OracleFactors:
    N: int
    nb: int
    F: np.ndarray            # factored matrix, N x N column-major
    ipiv: np.ndarray         # int32[N]
    Tq: np.ndarray           # n*n blocks of nb x nb
    dec: np.ndarray          # int8[n], 1 = LU
    s: np.ndarray
    m: np.ndarray
    margin: np.ndarray
    diag: np.ndarray         # see DG_*
    Bt: np.ndarray | None = None   # forward-transformed B in augmented mode
    domain: int = 0          # stride p of the diagonal domain (0: the diagonal tile alone)
    variant: int = 1         # LU-step variant: 1 = A1 (Alg. 2), 2 = A2 (Sec. 2.3)
    tree: int = 0            # QR elimination tree: 0 flat TS; S > 0 TS groups of S, TT tree over their heads
    Tt: np.ndarray | None = None  # TT factors of the killed heads (tree > 0)
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return (self.N + self.nb - 1) // self.nb

    def solve(self, B):
        return solve(self, B)


def factor(A, nb, criterion="max", alpha=1.0, seed=0, forced=None, mumps_reading=0,
           nsteps=-1, B=None, domain=0, estimate=False, variant=1, tree=0) -> OracleFactors:
    """Hybrid LU-QR factorization (Alg. 1) of a copy of A.  domain = p > 0
    pivots the LU attempt over the diagonal domain (the panel tiles k, k+p,
    k+2p, ...; Sec. 2.1), domain = 0 within the diagonal tile.  estimate:
    the criteria take ||A_kk^{-1}||_1 from the O(n_b^2) iterative estimate
    (Sec. 3.4) instead of computing it exactly.  variant: the LU step, 1 =
    A1 (GEPP on a backup of A_kk, Alg. 2), 2 = A2 (GEQRT of A_kk first, kept
    by a QR step; Sec. 2.3).  tree: the QR steps' elimination tree, 0 = flat
    TS (Alg. 4a), S > 0 = TS within groups of S tiles and a binary TT tree over
    the groups' heads (Alg. 3, 4a/4b; Sec. 2.2)."""
    A = _fortran(A)
    N = A.shape[0]
    assert A.shape == (N, N)
    n = (N + nb - 1) // nb
    crit = CRITERIA[criterion] if isinstance(criterion, str) else int(criterion)
    ipiv = np.zeros(N, dtype=np.int32)
    Tq = np.zeros(n * n * nb * nb, dtype=np.float64)
    dec = np.zeros(n, dtype=np.int8)
    s = np.zeros(n)
    m = np.zeros(n)
    margin = np.zeros(n)
    diag = np.zeros(DG_COUNT)
    f = None
    if forced is not None:
        f = np.ascontiguousarray(np.asarray(forced, dtype=np.int8))
        assert f.size >= n
    Bt = None
    nrhs = 0
    if B is not None:
        Bt = _fortran(B.reshape(N, -1) if B.ndim == 1 else B)
        nrhs = Bt.shape[1]
    Tt = np.zeros(n * n * nb * nb, dtype=np.float64) if tree else None
    if estimate or variant != 1 or tree:
        rc = lib().oracle_factor_t(N, _d(A), N, nb, crit, float(alpha), C.c_uint64(seed), _b(f),
                                   int(mumps_reading), int(nsteps), _d(Bt), N, nrhs, _i(ipiv), _d(Tq),
                                   _b(dec), _d(s), _d(m), _d(margin), _d(diag), int(domain),
                                   1 if estimate else 0, int(variant), int(tree), _d(Tt))
    elif domain:
        rc = lib().oracle_factor_domain(N, _d(A), N, nb, crit, float(alpha), C.c_uint64(seed), _b(f),
                                        int(mumps_reading), int(nsteps), _d(Bt), N, nrhs, _i(ipiv), _d(Tq),
                                        _b(dec), _d(s), _d(m), _d(margin), _d(diag), int(domain))
    else:
        rc = lib().oracle_factor(N, _d(A), N, nb, crit, float(alpha), C.c_uint64(seed), _b(f),
                                 int(mumps_reading), int(nsteps), _d(Bt), N, nrhs, _i(ipiv), _d(Tq),
                                 _b(dec), _d(s), _d(m), _d(margin), _d(diag))
    if rc != 0:
        raise ValueError(f"oracle_factor rejected argument {-rc}")
    return OracleFactors(N, nb, A, ipiv, Tq, dec, s, m, margin, diag, Bt, int(domain), int(variant), int(tree), Tt)


def solve(fac: OracleFactors, B):
    """Second-pass solve (Sec. 2.4): replay transforms on B, back-substitute."""
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    X = _fortran(B.reshape(fac.N, -1))
    if fac.tree:
        lib().oracle_solve_t(fac.N, _d(fac.F), fac.N, fac.nb, _i(fac.ipiv), _d(fac.Tq), _b(fac.dec),
                             _d(X), fac.N, X.shape[1], fac.domain, fac.variant, fac.tree, _d(fac.Tt))
    elif fac.variant == 2:
        lib().oracle_solve_v(fac.N, _d(fac.F), fac.N, fac.nb, _i(fac.ipiv), _d(fac.Tq), _b(fac.dec),
                             _d(X), fac.N, X.shape[1], fac.domain, 2)
    elif fac.domain:
        lib().oracle_solve_domain(fac.N, _d(fac.F), fac.N, fac.nb, _i(fac.ipiv), _d(fac.Tq), _b(fac.dec),
                                  _d(X), fac.N, X.shape[1], fac.domain)
    else:
        lib().oracle_solve(fac.N, _d(fac.F), fac.N, fac.nb, _i(fac.ipiv), _d(fac.Tq), _b(fac.dec),
                           _d(X), fac.N, X.shape[1])
    return X[:, 0] if vec else X


def forward(fac: OracleFactors, B):
    X = _fortran(np.asarray(B, dtype=np.float64).reshape(fac.N, -1))
    lib().oracle_forward_t(fac.N, _d(fac.F), fac.N, fac.nb, _i(fac.ipiv), _d(fac.Tq), _b(fac.dec),
                           _d(X), fac.N, X.shape[1], fac.domain, fac.variant, fac.tree, _d(fac.Tt))
    return X


def backward(fac: OracleFactors, Y):
    X = _fortran(np.asarray(Y, dtype=np.float64).reshape(fac.N, -1))
    lib().oracle_backward(fac.N, _d(fac.F), fac.N, fac.nb, _d(X), fac.N, X.shape[1])
    return X


# ---- tile-level routines (unit pins) ---------------------------------------

def gepp(W):
    W = _fortran(W)
    m = W.shape[0]
    ipiv = np.zeros(m, dtype=np.int32)
    z = lib().oracle_gepp(m, _d(W), m, _i(ipiv))
    return W, ipiv, int(z)


def inv_norm1(LU, ipiv):
    LU = _fortran(LU)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    return lib().oracle_inv_norm1(LU.shape[0], _d(LU), LU.shape[0], _i(ipiv))


def inv_norm1_est(LU):
    """O(m^2)-per-iteration estimate of ||W^{-1}||_1 from the factors L\\U of P W
    (Sec. 3.4; the permutation does not change the 1-norm)."""
    LU = _fortran(LU)
    return lib().oracle_inv_norm1_est(LU.shape[0], _d(LU), LU.shape[0])


def inv_norm1_qr(VR, T):
    """||A^{-1}||_1 from the GEQRT factors of A (V\\R and T; variant A2, Sec. 2.3)."""
    VR = _fortran(VR)
    T = _fortran(T)
    return lib().oracle_inv_norm1_qr(VR.shape[0], _d(VR), VR.shape[0], _d(T), T.shape[0])


def tile_norm1(A):
    A = _fortran(A)
    return lib().oracle_tile_norm1(_d(A), A.shape[0], A.shape[0], A.shape[1])


def geqrt(A):
    A = _fortran(A)
    m = A.shape[0]
    T = np.zeros((m, m), order="F")
    lib().oracle_geqrt(m, _d(A), m, _d(T), m)
    return A, T


def unmqr(V, T, Cm):
    V = _fortran(V)
    T = _fortran(T)
    Cm = _fortran(Cm)
    lib().oracle_unmqr(V.shape[0], _d(V), V.shape[0], _d(T), T.shape[0], Cm.shape[1], _d(Cm), Cm.shape[0])
    return Cm


def tsqrt(R, A):
    R = _fortran(R)
    A = _fortran(A)
    mk = R.shape[0]
    T = np.zeros((mk, mk), order="F")
    lib().oracle_tsqrt(mk, _d(R), mk, A.shape[0], _d(A), A.shape[0], _d(T), mk)
    return R, A, T


def tsmqr(Y, T, Ck, Ci):
    Y = _fortran(Y)
    T = _fortran(T)
    Ck = _fortran(Ck)
    Ci = _fortran(Ci)
    lib().oracle_tsmqr(Ck.shape[0], Ci.shape[0], _d(Y), Y.shape[0], _d(T), T.shape[0], Ck.shape[1],
                       _d(Ck), Ck.shape[0], _d(Ci), Ci.shape[0])
    return Ck, Ci


def ttqrt(R1, R2):
    """TTQRT of two upper-triangular tiles (Alg. 4b): returns R1', the tails Y
    (upper triangle of R2'), T."""
    R1 = _fortran(R1)
    R2 = _fortran(R2)
    m = R1.shape[0]
    T = np.zeros((m, m), order="F")
    lib().oracle_ttqrt(m, _d(R1), m, _d(R2), m, _d(T), m)
    return R1, R2, T


def ttmqr(Y, T, C1, C2):
    Y = _fortran(Y)
    T = _fortran(T)
    C1 = _fortran(C1)
    C2 = _fortran(C2)
    m = Y.shape[0]
    lib().oracle_ttmqr(m, _d(Y), m, _d(T), m, C1.shape[1], _d(C1), m, _d(C2), m)
    return C1, C2


def splitmix64(seed, k):
    return int(lib().oracle_splitmix64(C.c_uint64(seed), C.c_uint64(k)))


def uniform(seed, k):
    return float(lib().oracle_uniform(C.c_uint64(seed), C.c_uint64(k)))


def true_flops(N, nb, dec):
    d = np.ascontiguousarray(dec, dtype=np.int8)
    return lib().oracle_true_flops(N, nb, _b(d))


def num_threads():
    return int(lib().oracle_num_threads())


# ---- metrics of Sec. 5.1 ----------------------------------------------------

def hpl3(A, x, b):
    """HPL3 = ||Ax-b||_inf / (||A||_inf ||x||_inf eps N), eps = 2^-53 (Sec. 5.1)."""
    A = np.asarray(A)
    r = A @ x - b
    N = A.shape[0]
    return float(np.max(np.abs(r)) / (np.max(np.sum(np.abs(A), axis=1)) * np.max(np.abs(x)) * 2.0**-53 * N))


def backward_error(A, x, b):
    """eta = ||b - Ax||_inf / (||A||_inf ||x||_inf)."""
    A = np.asarray(A)
    r = b - A @ x
    return float(np.max(np.abs(r)) / (np.max(np.sum(np.abs(A), axis=1)) * np.max(np.abs(x))))
