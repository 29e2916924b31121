"""Seeded synthetic inputs for the hybrid LU-QR solver.

This module only draws matrices and right-hand sides; it holds none of the
solver's arithmetic, and both the HIP path's tests/benchmark and the CPU
oracle's tests take their inputs from here.

Every generator takes an explicit seed tuple and uses numpy's PCG64 seeded
through ``SeedSequence`` so that the same call gives the same bytes anywhere.
Matrices are float64, column-major (Fortran order), N x N.

Matrix types (the paper's workloads, Sec. 5.2 and Sec. 3.1):
  * ``gaussian``      iid N(0,1) ("random matrices" of Sec. 5.2).
  * ``diag_dominant`` N(0,1) + N I: column diagonally dominant in expectation.
  * ``growth_prone``  the growth example of Sec. 3.1 at alpha = 1: 1 on the
                      diagonal, -1 strictly below, 1 in the last column, plus a
                      1e-8 N(0,1) perturbation.
  * ``kron_example``  the same example lifted to tiles, M (x) I_nb, where M has
                      1/alpha on the diagonal (last entry 1), -1 below it and 1
                      in the last column.
  * ``usv``           U diag(sigma) V^T with U, V Haar-orthogonal and sigma
                      log-spaced from 1 to 1/kappa.
"""
from __future__ import annotations

import numpy as np

TYPES = ("gaussian", "diag_dominant", "growth_prone", "usv")


def rng(*seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(s) for s in seed])))


def gaussian(N, seed=(0,)):
    return np.asfortranarray(rng(1, *seed, N).standard_normal((N, N)))


def diag_dominant(N, seed=(0,)):
    A = rng(2, *seed, N).standard_normal((N, N))
    A[np.diag_indices(N)] += N
    return np.asfortranarray(A)


def growth_prone(N, seed=(0,), perturb=1e-8):
    A = -np.tril(np.ones((N, N)), -1)
    A[np.diag_indices(N)] = 1.0
    A[:, -1] = 1.0
    if perturb:
        A = A + perturb * rng(3, *seed, N).standard_normal((N, N))
    return np.asfortranarray(A)


def kron_example(n, nb, alpha):
    M = -np.tril(np.ones((n, n)), -1)
    M[np.diag_indices(n)] = 1.0 / alpha
    M[:, -1] = 1.0
    return np.asfortranarray(np.kron(M, np.eye(nb)))


def mumps_example(nb=3):
    """Two tile rows of size nb >= 3 whose first panel separates readings of
    the MUMPS estimate (Sec. 3.3).  The leading 3 x 3 block of A_00 is
    [[4, 2, 2], [2, 5, 3], [0, 2, 4]] and the rest of A_00 is 8 I; A_10 holds
    diag(1, -4, 5) in its leading 3 x 3 block and zeros elsewhere; A_01 = 0
    and A_11 = 10 I.  The hand computation of the step-0 criterion is written
    out in the oracle test that uses it."""
    assert nb >= 3
    A = np.zeros((2 * nb, 2 * nb))
    A[:3, :3] = [[4.0, 2.0, 2.0], [2.0, 5.0, 3.0], [0.0, 2.0, 4.0]]
    A[3:nb, 3:nb] = 8.0 * np.eye(nb - 3)
    A[nb:nb + 3, :3] = np.diag([1.0, -4.0, 5.0])
    A[nb:, nb:] = 10.0 * np.eye(nb)
    return np.asfortranarray(A)


def haar(N, g: np.random.Generator):
    """Haar-distributed orthogonal matrix: Q of a Gaussian with diag(R) > 0 (Mezzadri 2007)."""
    Z = g.standard_normal((N, N))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))


def sigmas(N, kappa):
    i = np.arange(N, dtype=np.float64)
    return kappa ** (-i / max(N - 1, 1))


def usv(N, kappa, seed=(0,)):
    g = rng(4, *seed, N, int(round(np.log10(kappa) * 1000)))
    U = haar(N, g)
    V = haar(N, g)
    return np.asfortranarray((U * sigmas(N, kappa)) @ V.T)


HAAR_MAX_ELEMENTS = 2 ** 31 - 1  # largest N x N for which the device QR gives an orthogonal factor


def usv_torch(N, kappa, seed=(0,), device="cuda"):
    """Same construction drawn with torch on a device (large N only).

    The Gaussian factors come from torch's own generator seeded from the seed
    tuple, so the matrix differs from ``usv`` at the same seed but is
    reproducible from run to run.
    """
    import torch
    ss = np.random.SeedSequence([5, *[int(s) for s in seed], N, int(round(np.log10(kappa) * 1000))])
    gen = torch.Generator(device=device)
    gen.manual_seed(int(ss.generate_state(1, dtype=np.uint64)[0] & ((1 << 63) - 1)))

    def _haar(n):
        Z = torch.randn(n, n, generator=gen, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(Z)
        Q *= torch.sign(torch.diagonal(R)).unsqueeze(0)
        return Q

    def _orthogonal():
        if N * N <= HAAR_MAX_ELEMENTS:
            return _haar(N)
        # The device QR returns a non-orthogonal Q once an N x N array passes
        # 2^31 elements (measured: ||Q^T Q - I|| ~ 5e4 at N = 47104), so larger
        # factors are built as D1 P D2 with D1, D2 block-diagonal of two Haar
        # blocks each and P a random permutation: exactly orthogonal, with
        # every column mixed across both halves.
        h = N // 2
        Q = torch.zeros(N, N, device=device, dtype=torch.float64)
        Q[:h, :h] = _haar(h)
        Q[h:, h:] = _haar(N - h)
        perm = torch.randperm(N, generator=gen, device=device)
        D2 = torch.zeros(N, N, device=device, dtype=torch.float64)
        D2[:h, :h] = _haar(h)
        D2[h:, h:] = _haar(N - h)
        Q = Q[:, perm] @ D2
        return Q

    U = _orthogonal()
    V = _orthogonal()
    s = torch.as_tensor(sigmas(N, kappa), device=device)
    A = (U * s.unsqueeze(0)) @ V.T.contiguous()
    del U, V
    return A.T.contiguous().T  # column-major storage (stride (1, N))


def matrix(kind, N, seed=(0,), kappa=None):
    if kind == "gaussian":
        return gaussian(N, seed)
    if kind == "diag_dominant":
        return diag_dominant(N, seed)
    if kind == "growth_prone":
        return growth_prone(N, seed)
    if kind == "usv":
        return usv(N, kappa, seed)
    raise ValueError(kind)


def rhs(N, nrhs=1, seed=(0,)):
    B = rng(6, *seed, N, nrhs).standard_normal((N, nrhs))
    return np.asfortranarray(B[:, 0] if nrhs == 1 else B)
