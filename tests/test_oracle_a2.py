"""Pins of the oracle's LU-step variant A2 (Sec. 2.3: the diagonal tile is
QR-factored first; an LU step eliminates with its triangular factor U and
applies Q^T to the tiles on its right; a QR step continues from the same
factorization, so no backup is kept).

What fixes the answer independently of the oracle:
  * ||A_kk^{-1}||_1 from the QR factors equals the 1-norm of numpy's inverse
    and of the A1 route (GEPP factors), three different computations;
  * the Factor is LAPACK's QR (scipy, same sign convention): R must match;
  * one A2 LU step leaves the Schur complement A22 - A21 A11^{-1} A12 in the
    trailing tiles (numpy solve), L_ik = A_ik R^{-1} and U_kj = Q^T A_kj with
    LAPACK's Q and R;
  * an all-QR sequence is the same computation in both variants (bitwise);
  * every forced sequence on a small matrix solves A x = b to rounding
    (brute force over all 2^n sequences, ragged last tile included);
  * the criterion sees the same A_kk as in A1, so decisions away from ties
    agree with A1's and s_k = 1/||A_kk^{-1}||_1 agrees to rounding;
  * Tab. 1 work: the Factor and the Apply of an A2 LU step cost twice A1's.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_5522_amd import inputs


def _forced(seq):
    return np.asarray(seq, dtype=np.int8)


@pytest.mark.parametrize("m", [1, 2, 5, 16, 64])
def test_inv_norm1_from_qr_factors(O, m):
    rng = np.random.default_rng(900 + m)
    for t in range(4):
        A = rng.standard_normal((m, m)) * np.exp(rng.uniform(-2, 2, size=(1, m)))
        VR, T = O.geqrt(A.copy())
        got = O.inv_norm1_qr(VR, T)
        ref = np.linalg.norm(np.linalg.inv(A), 1)
        W, piv, z = O.gepp(A.copy())
        assert z == 0
        assert got == pytest.approx(ref, rel=1e-10)
        assert got == pytest.approx(O.inv_norm1(W, piv), rel=1e-10)


def test_a2_factor_is_lapack_qr(O):
    rng = np.random.default_rng(910)
    N, nb = 48, 16
    A = rng.standard_normal((N, N))
    f = O.factor(A, nb, "forced", forced=_forced([1, 1, 1]), nsteps=1, variant=2)
    R = sla.qr(A[:nb, :nb], mode="r")[0]
    got = np.triu(f.F[:nb, :nb])
    assert np.allclose(got, R, rtol=0, atol=1e-12 * np.abs(R).max())


def test_a2_lu_step_leaves_schur_complement(O):
    rng = np.random.default_rng(911)
    N, nb = 60, 16  # ragged last tile (12 rows)
    A = rng.standard_normal((N, N))
    f = O.factor(A, nb, "forced", forced=_forced([1, 0, 0, 0]), nsteps=1, variant=2)
    A11, A12, A21, A22 = A[:nb, :nb], A[:nb, nb:], A[nb:, :nb], A[nb:, nb:]
    S = A22 - A21 @ np.linalg.solve(A11, A12)
    assert np.allclose(f.F[nb:, nb:], S, rtol=0, atol=1e-11 * np.abs(S).max())
    Q, R = sla.qr(A11)
    L = np.linalg.solve(R.T, A21.T).T  # A21 R^{-1}
    assert np.allclose(f.F[nb:, :nb], L, rtol=0, atol=1e-11 * np.abs(L).max())
    U = Q.T @ A12
    assert np.allclose(f.F[:nb, nb:], U, rtol=0, atol=1e-11 * np.abs(U).max())
    assert f.dec[0] == 1
    assert np.array_equal(f.ipiv[:nb], np.arange(nb))


def test_a2_all_qr_is_a1_all_qr(O):
    rng = np.random.default_rng(912)
    N, nb = 64, 16
    A = rng.standard_normal((N, N))
    b = rng.standard_normal(N)
    seq = _forced([0, 0, 0, 0])
    f1 = O.factor(A, nb, "forced", forced=seq, variant=1)
    f2 = O.factor(A, nb, "forced", forced=seq, variant=2)
    assert np.array_equal(f1.F, f2.F)
    assert np.array_equal(f1.Tq, f2.Tq)
    assert np.array_equal(f1.solve(b), f2.solve(b))


@pytest.mark.parametrize("N,nb", [(32, 8), (29, 8)])
def test_a2_every_forced_sequence_solves(O, N, nb):
    rng = np.random.default_rng(913 + N)
    A = rng.standard_normal((N, N))
    b = rng.standard_normal(N)
    xref = np.linalg.solve(A, b)
    n = (N + nb - 1) // nb
    for seq in itertools.product([0, 1], repeat=n):
        f = O.factor(A, nb, "forced", forced=_forced(seq), variant=2)
        assert list(f.dec) == list(seq)
        x = f.solve(b)
        assert np.linalg.norm(x - xref) <= 1e-10 * np.linalg.norm(xref), seq


def test_a2_augmented_rhs_matches_forward_replay(O):
    rng = np.random.default_rng(914)
    N, nb = 80, 16
    A = rng.standard_normal((N, N))
    B = rng.standard_normal((N, 3))
    f = O.factor(A, nb, "forced", forced=_forced([1, 0, 1, 1, 0]), B=B, variant=2)
    Y = O.forward(f, B)
    assert np.allclose(f.Bt, Y, rtol=0, atol=1e-12 * np.abs(Y).max())


@pytest.mark.parametrize("crit,alpha", [("max", 1.0), ("max", 8.0), ("sum", 2.0), ("sum", 40.0)])
def test_a2_decisions_agree_with_a1(O, crit, alpha):
    N, nb = 128, 16
    A = inputs.gaussian(N, seed=(915,))
    f1 = O.factor(A, nb, crit, alpha, variant=1)
    f2 = O.factor(A, nb, crit, alpha, variant=2)
    assert 0 < f1.dec.sum() < f1.n  # a hybrid sequence
    k = 0
    while k < f1.n and f1.dec[k] == f2.dec[k]:
        # the same decisions so far: both variants left the same trailing matrix
        # (an LU step leaves the Schur complement either way), so the criterion
        # inputs agree to rounding
        assert f2.s[k] == pytest.approx(f1.s[k], rel=1e-9)
        assert f2.m[k] == pytest.approx(f1.m[k], rel=1e-9)
        k += 1
    if k < f1.n:  # the first difference must be a tie of the criterion
        assert abs(f1.margin[k]) < 1e-6, (k, f1.margin[k], f2.margin[k])


def test_a2_singular_tile_info(O):
    rng = np.random.default_rng(916)
    N, nb = 48, 16
    A = rng.standard_normal((N, N))
    A[:nb, 5] = 0.0  # column 5 of A_00 is zero: U_00(5,5) = 0 and the tile is singular
    f = O.factor(A, nb, "max", 1.0, variant=2)
    assert f.dec[0] == 0 and f.s[0] == 0.0
    f = O.factor(A, nb, "max", np.inf, variant=2)
    assert f.dec[0] == 1
    assert f.diag[O.DG_INFO] == 6  # 1-based row of the first zero on U's diagonal
    g = O.factor(A, nb, "max", np.inf, variant=1)
    assert g.diag[O.DG_INFO] == f.diag[O.DG_INFO]


def test_a2_rejected_combinations(O):
    A = np.eye(32)
    for kw in (dict(criterion="mumps"), dict(domain=1), dict(estimate=True)):
        with pytest.raises(ValueError, match="23"):
            O.factor(A, 8, variant=2, **kw)
    with pytest.raises(ValueError, match="22"):
        O.factor(A, 8, variant=3)


def test_a2_true_flops(O):
    rng = np.random.default_rng(917)
    N, nb = 64, 16
    n = N // nb
    A = rng.standard_normal((N, N))
    lu = O.factor(A, nb, "forced", forced=_forced([1] * n), variant=2)
    want = sum(4 / 3 + 3 * r + 2 * r * r for r in range(n - 1, -1, -1)) * nb ** 3
    assert lu.diag[O.DG_TRUEFLOPS] == pytest.approx(want, rel=1e-12)
    qr1 = O.factor(A, nb, "forced", forced=_forced([0] * n), variant=1)
    qr2 = O.factor(A, nb, "forced", forced=_forced([0] * n), variant=2)
    assert qr2.diag[O.DG_TRUEFLOPS] == qr1.diag[O.DG_TRUEFLOPS]
