"""Torch-facing façade over the C ABI: device memory and the current stream
come from PyTorch, every step of the factorization and solve runs in the HIP
kernels of libluqr.so (see include/luqr.h for the contract of each call).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor(A: torch.Tensor) -> torch.Tensor:
    """Column-major float64 device copy/view of a 2-D A: element (i, j) at
    data_ptr + i + j*A.shape[0] (leading dimension = number of rows)."""
    A = A.to(device="cuda", dtype=torch.float64)
    if A.dim() == 1:
        A = A.reshape(-1, 1)
    rows, cols = A.shape
    if (cols == 1 and A.is_contiguous()) or (A.stride(0) == 1 and A.stride(1) == rows):
        return A
    out = torch.empty((cols, rows), dtype=torch.float64, device="cuda").t()
    out.copy_(A)
    return out


class Factors:
    """Handle of one hybrid LU-QR factorization (Alg. 1)."""

    def __init__(self, A, nb, criterion="max", alpha=1.0, precision="fp64", nrhs_max=1, seed=0,
                 forced=None, nsteps=-1, mumps_reading=0, timing=False, work=None):
        A = colmajor(A)
        self.N = N = A.shape[0]
        self._lda = N
        self.nb = nb
        self.n = (N + nb - 1) // nb
        self.precision = precision
        self.opts, self._keep = L.make_opts(nb, criterion, alpha, precision, nrhs_max, seed, forced, nsteps,
                                            mumps_reading, timing)
        nbytes = L.luqr_workspace_bytes(N, self.opts)
        if work is None or work.numel() < nbytes + 256:
            work = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        self.work = work
        base = self.work.data_ptr()
        off = (-base) % 256
        self._wptr = C.c_void_p(base + off)
        self._wbytes = nbytes
        self.h = L.luqr_factor(N, C.c_void_p(A.data_ptr()), N, self.opts, self._wptr, nbytes, _stream())

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                L.luqr_destroy(h)
            except Exception:
                pass
            self.h = None

    def solve(self, B: torch.Tensor) -> torch.Tensor:
        vec = B.dim() == 1
        Bm = B.reshape(self.N, -1)
        X = torch.empty((Bm.shape[1], self.N), dtype=torch.float64, device="cuda").t()
        X.copy_(Bm)
        L.luqr_solve(self.h, X.shape[1], C.c_void_p(X.data_ptr()), self.N, _stream())
        return X[:, 0] if vec else X

    def solve_refined(self, A: torch.Tensor, B: torch.Tensor, max_iter=10) -> torch.Tensor:
        A = colmajor(A)
        vec = B.dim() == 1
        Bc = colmajor(B.reshape(self.N, -1))
        X = torch.empty((Bc.shape[1], self.N), dtype=torch.float64, device="cuda").t()
        L.luqr_solve_refined(self.h, C.c_void_p(A.data_ptr()), self.N, Bc.shape[1],
                             C.c_void_p(Bc.data_ptr()), self.N, C.c_void_p(X.data_ptr()), self.N,
                             max_iter, _stream())
        return X[:, 0] if vec else X

    def decisions(self):
        n = self.n
        dec = np.zeros(n, np.int8)
        s = np.zeros(n)
        m = np.zeros(n)
        mg = np.zeros(n)
        L.luqr_get_decisions(self.h, dec.ctypes.data, s.ctypes.data, m.ctypes.data, mg.ctypes.data, n)
        return dec, s, m, mg

    def status(self):
        return L.luqr_get_status(self.h)

    PHASES = ("panel", "lu_apply", "lu_update", "qr_step", "qr_rinv")

    def step_times(self):
        """(n, 5) array of per-step phase durations in ms (columns: PHASES);
        needs timing=True at construction."""
        t = np.zeros((self.n, L.NPHASE), np.float32)
        L.luqr_get_step_times(self.h, t.ctypes.data, self.n)
        return t

    def export(self):
        F = torch.empty((self.N, self.N), dtype=torch.float64, device="cuda").t()  # column-major
        ipiv = np.zeros(self.N, np.int32)
        L.luqr_export_factors(self.h, C.c_void_p(F.data_ptr()), self.N, ipiv.ctypes.data, _stream())
        return F, ipiv


def factor(A, nb, **kw) -> Factors:
    return Factors(A, nb, **kw)
