"""Diagonal-domain pivoting (Sec. 2.1, last paragraph; Sec. 3.1; Sec. 3.3)
on the GPU against the FP64 oracle, through the C ABI.

The LU attempt of step k is GEPP on the stacked panel tiles k, k+p, k+2p, ...;
the criterion sees A_kk and the tiles below after its interchanges, and an
LU step interchanges the trailing columns of the domain's rows.  Bar as for
the tile variant: decisions equal outside a 1e-6 margin band, s_k and m_k to
1e-9, factors to 1e-10 of the largest entry with the pivots (stacked row
indices) equal, solutions to 1e-10; and p >= n gives the tile variant bit
for bit.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_5522_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_1401_5522_amd import solver
    return solver


def dev(a):
    import torch
    return torch.from_numpy(np.asfortranarray(a)).cuda()


CASES = [
    # (kind, N, nb, criterion, alpha, p)
    ("gaussian", 512, 64, "max", 100.0, 2),      # four tiles in the first domain
    ("gaussian", 512, 128, "max", 300.0, 3),
    ("gaussian", 1000, 128, "max", np.inf, 2),   # 512 stacked rows, ragged last tile, all LU
    ("gaussian", 320, 32, "mumps", 2.1, 1),      # the whole panel is the domain
    ("diag_dominant", 448, 64, "sum", 0.5, 2),
    ("gaussian", 384, 32, "max", 40.0, 4),
]


@pytest.mark.parametrize("kind,N,nb,crit,alpha,p", CASES)
def test_domain_fp64_parity(O, gpu, kind, N, nb, crit, alpha, p):
    A = inputs.matrix(kind, N, seed=(180, N))
    b = inputs.rhs(N, seed=(181, N))
    f = gpu.factor(dev(A), nb, criterion=crit, alpha=alpha, domain=p)
    dec, s, m, mg = f.decisions()
    F, ipiv = f.export()
    F = F.cpu().numpy()
    st = f.status()
    x = f.solve(dev(b)).cpu().numpy()
    o = O.factor(A, nb, crit, alpha, domain=p)
    assert st.watchdog == 0
    upto = len(o.dec)
    for k in range(len(o.dec)):
        if abs(o.margin[k]) <= 1e-6:
            upto = k
            break
        assert dec[k] == o.dec[k], (k, dec, o.dec, o.margin[k])
    assert (np.abs(s[:upto] - o.s[:upto]) <= 1e-9 * np.abs(o.s[:upto])).all()
    assert (np.abs(m[:upto] - o.m[:upto]) <= 1e-9 * np.maximum(np.abs(o.m[:upto]), 1e-300)).all()
    if upto == len(o.dec):
        assert np.abs(F - o.F).max() <= 1e-10 * max(np.abs(o.F).max(), 1.0)
        np.testing.assert_array_equal(ipiv, o.ipiv)
        xo = o.solve(b)
        assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)
    assert O.backward_error(A, x, b) <= N * 2.0 ** -53 * 10
    assert int(dec.sum()) > 0


def test_whole_panel_domain_is_lapack_getrf(gpu):
    N, nb = 256, 32
    A = inputs.gaussian(N, seed=(182,))
    f = gpu.factor(dev(A), nb, criterion="max", alpha=np.inf, domain=1)
    F, ipiv = f.export()
    F = F.cpu().numpy()
    lu, piv = sla.lu_factor(A)
    gp = np.array([k * nb + (ipiv[k * nb + c] // nb) * nb + ipiv[k * nb + c] % nb
                   for k in range(N // nb) for c in range(nb)])
    np.testing.assert_array_equal(gp, piv)
    assert np.abs(np.triu(F) - np.triu(lu)).max() <= 1e-12 * np.abs(lu).max()


def test_stride_beyond_panel_is_the_tile_variant(gpu):
    N, nb = 512, 64
    A = dev(inputs.gaussian(N, seed=(183,)))
    runs = []
    for p in (0, N // nb):
        f = gpu.factor(A, nb, criterion="max", alpha=200.0, domain=p)
        F, ipiv = f.export()
        runs.append((F.cpu().numpy(), ipiv, f.decisions()[0]))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    np.testing.assert_array_equal(runs[0][2], runs[1][2])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_domain_mixed_precision_refined(O, gpu, prec):
    N, nb, p, alpha = 1024, 128, 2, 1e4
    A = inputs.usv(N, 1e2, seed=(184, N))
    b = inputs.rhs(N, seed=(185, N))
    Ad = dev(A)
    f = gpu.factor(Ad, nb, criterion="max", alpha=alpha, precision=prec, domain=p)
    x = f.solve_refined(Ad, dev(b), max_iter=30).cpu().numpy()
    st = f.status()
    dec = f.decisions()[0]
    o = O.factor(A, nb, "max", alpha, domain=p)
    band = 1e-3 if prec == "fp32" else 2e-2
    for k in range(len(o.dec)):
        if abs(o.margin[k]) <= band:
            break
        assert dec[k] == o.dec[k], (k, dec, o.dec)
    assert st.watchdog == 0 and st.ir_converged == 1, (st.ir_iters, st.ir_eta)
    r = b - A @ x
    assert np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max()) <= N * 1e-16
