"""QR steps whose trailing matrix is wide enough that the QR-step grid (16
producers + 4 (n-k-1) consumer strips at n_b = 256) exceeds the CU count, so
that the kernel relies on two workgroups being resident per CU.  At
N = 16384, n_b = 256 this holds for the first steps; alpha = 0 makes every
step a QR step (Sec. 3).

The oracle does not reach this size, so the bar is the solution-level one of
the mixed-precision tests: refinement reaches backward error <= N 1e-16 in a
few passes (it would not with a wrong trailing update), and the refined
solution agrees with the FP64 GPU path (one workgroup per CU) within
4 cond N 1e-16 (cond bounded by N kappa for UΣV^T).
"""
import numpy as np
import pytest

from paper_1401_5522_amd import inputs

pytestmark = pytest.mark.gpu

N, NB, KAPPA = 16384, 256, 1e2


@pytest.fixture(scope="module")
def system():
    import torch
    assert torch.cuda.is_available()
    A = inputs.usv_torch(N, KAPPA, seed=(130,))
    b = torch.from_numpy(inputs.rhs(N, 1, seed=(131, N))).cuda()
    return A, b


def backward_error(A, x, b):
    r = b - A @ x
    return float(r.abs().max() / (A.abs().sum(dim=1).max() * x.abs().max()))


@pytest.fixture(scope="module")
def x64(system):
    from paper_1401_5522_amd import solver
    A, b = system
    f = solver.factor(A, NB, criterion="max", alpha=0.0, precision="fp64")
    x = f.solve(b)
    assert f.status().watchdog == 0
    assert backward_error(A, x, b) <= N * 1e-16
    return x


@pytest.mark.parametrize("prec,max_passes", [("fp32", 4), ("bf16", 40)])
def test_wide_qr_steps(system, x64, prec, max_passes):
    from paper_1401_5522_amd import solver
    A, b = system
    f = solver.factor(A, NB, criterion="max", alpha=0.0, precision=prec)
    dec = f.decisions()[0]
    assert (dec == 0).all()
    x = f.solve_refined(A, b, max_iter=max_passes)
    st = f.status()
    assert st.watchdog == 0
    assert st.ir_converged == 1 and st.ir_iters <= max_passes, (st.ir_iters, st.ir_eta)
    assert backward_error(A, x, b) <= N * 1e-16
    fwd = float((x - x64).abs().max() / x64.abs().max())
    assert fwd <= 4 * (N * KAPPA) * N * 1e-16, fwd
