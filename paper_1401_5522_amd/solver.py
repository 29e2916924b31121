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
                 forced=None, nsteps=-1, timing=False, work=None, lookahead=True, domain=0, estimate=False,
                 variant=1, tree=0):
        A = colmajor(A)
        self.N = N = A.shape[0]
        self._lda = N
        self.nb = nb
        self.n = (N + nb - 1) // nb
        self.precision = precision
        self.opts, self._keep = L.make_opts(nb, criterion, alpha, precision, nrhs_max, seed, forced, nsteps,
                                            timing, lookahead, domain, estimate, variant, tree)
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

    def solve_gmres_ir(self, A: torch.Tensor, b: torch.Tensor, max_outer=10, max_inner=30):
        """GMRES-based refinement of one right-hand side; returns (x, inner
        steps)."""
        A = colmajor(A)
        bc = b.reshape(-1).to(device="cuda", dtype=torch.float64).contiguous()
        x = torch.empty(self.N, dtype=torch.float64, device="cuda")
        inner = L.luqr_solve_gmres_ir(self.h, C.c_void_p(A.data_ptr()), self.N, C.c_void_p(bc.data_ptr()),
                                      C.c_void_p(x.data_ptr()), max_outer, max_inner, _stream())
        return x, inner

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


class Batch:
    """Many independent systems solved by the persistent batched kernel
    (luqr_batched_* in include/luqr.h): FP32 tiles, FP64 refinement, tile size
    32 or 64 per system.  `As` are 2-D FP64 device tensors (any layout; a
    column-major copy is kept), `nb` an int or one int per system.  Outputs
    live in self.X (one FP64 vector per system), self.dec, self.eta, self.iters;
    run() only enqueues, so it can be captured in a CUDA/HIP graph."""

    def __init__(self, As, nb=64, criterion="max", alpha=1.0, max_iter=10):
        self.A = [colmajor(A) for A in As]
        self.batch = B = len(self.A)
        self.N = np.array([A.shape[0] for A in self.A], np.int64)
        ld = self.N.copy()
        self.nb = np.array(nb if np.ndim(nb) else [nb] * B, np.int32)
        self.opts, self._keep = L.make_opts(int(self.nb[0]), criterion, alpha, "fp32", 1)
        nbytes = L.luqr_batched_workspace_bytes(B, self.N.ctypes.data, self.nb.ctypes.data, self.opts)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.work.data_ptr()
        self._wptr = C.c_void_p(base + (-base) % 256)
        self._wbytes = nbytes
        self.plan = L.luqr_batched_plan(B, self.N.ctypes.data, self.nb.ctypes.data, ld.ctypes.data, ld.ctypes.data,
                                        ld.ctypes.data, self.opts, max_iter, self._wptr, nbytes)
        self.X = [torch.zeros(int(n), dtype=torch.float64, device="cuda") for n in self.N]
        self.stride = L.luqr_batched_decision_stride(self.plan)
        self.dec = torch.full((B * self.stride,), -1, dtype=torch.int8, device="cuda")
        self.eta = torch.zeros(B, dtype=torch.float64, device="cuda")
        self.iters = torch.zeros(B, dtype=torch.int32, device="cuda")
        self._pA = torch.tensor([A.data_ptr() for A in self.A], dtype=torch.int64, device="cuda")
        self._pX = torch.tensor([x.data_ptr() for x in self.X], dtype=torch.int64, device="cuda")
        self._pB = None
        self.Bs = None

    def set_rhs(self, Bs):
        self.Bs = [b.to(device="cuda", dtype=torch.float64).contiguous() for b in Bs]
        self._pB = torch.tensor([b.data_ptr() for b in self.Bs], dtype=torch.int64, device="cuda")

    def run(self):
        L.luqr_batched_run(self.plan, C.c_void_p(self._pA.data_ptr()), C.c_void_p(self._pB.data_ptr()),
                           C.c_void_p(self._pX.data_ptr()), C.c_void_p(self.dec.data_ptr()),
                           C.c_void_p(self.eta.data_ptr()), C.c_void_p(self.iters.data_ptr()), _stream())

    def decisions(self):
        d = self.dec.view(self.batch, self.stride).cpu().numpy()
        return [d[s, : (int(self.N[s]) + int(self.nb[s]) - 1) // int(self.nb[s])] for s in range(self.batch)]

    def __del__(self):
        p = getattr(self, "plan", None)
        if p:
            try:
                L.luqr_batched_destroy(p)
            except Exception:
                pass
            self.plan = None


def batched_autotune(As, Bs, criterion="max", alpha=1.0, max_iter=10, sample=32):
    """Tile size per system chosen by luqr_batched_autotune (timed on the
    device per size class); returns (nb array, timings [class][nb 32, nb 64] in ms)."""
    A = [colmajor(a) for a in As]
    Bv = [b.to(device="cuda", dtype=torch.float64).contiguous() for b in Bs]
    B = len(A)
    N = np.array([a.shape[0] for a in A], np.int64)
    ld = N.copy()
    opts, keep = L.make_opts(64, criterion, alpha, "fp32", 1)
    n64 = np.full(B, 64, np.int32)
    n32 = np.full(B, 32, np.int32)
    nbytes = max(L.luqr_batched_workspace_bytes(B, N.ctypes.data, n64.ctypes.data, opts),
                 L.luqr_batched_workspace_bytes(B, N.ctypes.data, n32.ctypes.data, opts)) + 24 * B + 4096
    work = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = work.data_ptr()
    wptr = C.c_void_p(base + (-base) % 256)
    X = [torch.zeros(int(n), dtype=torch.float64, device="cuda") for n in N]
    pA = torch.tensor([a.data_ptr() for a in A], dtype=torch.int64, device="cuda")
    pB = torch.tensor([b.data_ptr() for b in Bv], dtype=torch.int64, device="cuda")
    pX = torch.tensor([x.data_ptr() for x in X], dtype=torch.int64, device="cuda")
    nb_out = np.zeros(B, np.int32)
    ms = np.zeros(12, np.float32)
    L.luqr_batched_autotune(B, N.ctypes.data, ld.ctypes.data, ld.ctypes.data, ld.ctypes.data, opts, max_iter,
                            C.c_void_p(pA.data_ptr()), C.c_void_p(pB.data_ptr()), C.c_void_p(pX.data_ptr()),
                            sample, wptr, nbytes, _stream(), nb_out.ctypes.data, ms.ctypes.data)
    return nb_out, ms.reshape(6, 2)
