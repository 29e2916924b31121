"""luqr_solve_noalloc (the entry point that allocates nothing: its workspace
is the library's own per-GPU device buffer) against luqr_factor +
luqr_solve_refined on a workspace the caller allocates, through the C ABI.

Two calls in a row share the one buffer, the second with a smaller system,
so anything the second call needed cleared and did not clear would show.
Both paths run the same kernels in the same order (the reference runs
without lookahead, as the no-allocation path does), so the results are
expected to agree to rounding of identical operations; the bar is a
normwise relative difference of 1e-12 and equal decision counts and
refinement iterations.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1401_5522_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    # (matrix, N, nb, precision, alpha, nrhs): the second is smaller than the first
    ("usv", 1000, 128, "fp32", 1e4, 2),
    ("gaussian", 300, 64, "fp64", 60.0, 1),
]


def _reference(A, B, nb, prec, alpha, max_iter):
    """luqr_factor + luqr_solve_refined with a caller-provided workspace."""
    import torch
    from paper_1401_5522_amd import _lib as L
    N, nrhs = B.shape
    o, keep = L.make_opts(nb, "max", alpha, prec, nrhs_max=nrhs, lookahead=False)
    nbytes = L.luqr_workspace_bytes(N, o)
    work = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (work.data_ptr() + 255) // 256 * 256
    X = torch.empty_like(B)
    h = L.luqr_factor(N, A.data_ptr(), N, o, base, nbytes, None)
    try:
        L.luqr_solve_refined(h, A.data_ptr(), N, nrhs, B.data_ptr(), N, X.data_ptr(), N, max_iter, None)
        st = L.luqr_get_status(h)
    finally:
        L.luqr_destroy(h)
    torch.cuda.synchronize()
    return X, st


def test_noalloc_matches_allocating_path_twice():
    import torch
    from paper_1401_5522_amd import _lib as L
    assert torch.cuda.is_available()
    for kind, N, nb, prec, alpha, nrhs in CASES:
        print(f"noalloc case {kind} N={N} nb={nb} {prec} alpha={alpha:g} nrhs={nrhs}", flush=True)
        A0 = inputs.usv(N, 1e2, seed=(170, N)) if kind == "usv" else inputs.gaussian(N, seed=(171, N))
        A = torch.from_numpy(A0).cuda()
        B = torch.from_numpy(np.asfortranarray(inputs.rhs(N, nrhs, seed=(172, N)).reshape(N, nrhs))).cuda()
        B = B.t().contiguous().t()
        Xr, sr = _reference(A, B, nb, prec, alpha, 10)
        o, keep = L.make_opts(nb, "max", alpha, prec, nrhs_max=nrhs)
        assert L.luqr_workspace_bytes(N, o) <= L.NOALLOC_SCRATCH_BYTES
        X = torch.full_like(B, float("nan"))
        st = L.luqr_solve_noalloc(N, A.data_ptr(), N, o, nrhs, B.data_ptr(), N, X.data_ptr(), N, 10, None)
        torch.cuda.synchronize()
        assert st.watchdog == 0 and sr.watchdog == 0
        assert st.n_lu == sr.n_lu and st.ir_iters == sr.ir_iters and st.ir_converged == sr.ir_converged == 1
        assert st.ir_eta <= N * 1e-16
        rel = float(torch.linalg.norm(X - Xr) / torch.linalg.norm(Xr))
        assert rel <= 1e-12, rel


def test_noalloc_rejects_what_does_not_fit():
    from paper_1401_5522_amd import _lib as L
    N = 4096
    o, keep = L.make_opts(128, "max", 1.0, "fp64")
    assert L.luqr_workspace_bytes(N, o) > L.NOALLOC_SCRATCH_BYTES
    st = L.luqr_status()
    rc = L.lib().luqr_solve_noalloc(N, C.c_void_p(256), N, C.byref(o), 1, C.c_void_p(256), N, C.c_void_p(256), N,
                                    0, C.byref(st), None)
    assert rc == L.LUQR_ERR_TOO_LARGE
    o.timing = 1
    rc = L.lib().luqr_solve_noalloc(256, C.c_void_p(256), 256, C.byref(o), 1, C.c_void_p(256), 256,
                                    C.c_void_p(256), 256, 0, C.byref(st), None)
    assert rc == -4
