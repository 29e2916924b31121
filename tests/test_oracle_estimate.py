"""Pins of the oracle's O(n_b^2) estimate of ||A_kk^{-1}||_1 (Sec. 3.4: the
inverse norm approximated from the L and U factors by an iterative method).

What fixes the answer independently of the oracle:
  * LAPACK's condition estimator (dgecon through scipy) runs the same
    Hager-Higham iteration on the same factors with its own triangular
    solves: 1 / (rcond ||A||_1) must equal the estimate to rounding;
  * every iterate is ||B x||_1 with ||x||_1 <= 1, so the estimate is a lower
    bound of the exact norm (computed column by column);
  * closed forms where the iteration is exact: n = 1; a diagonal matrix (the
    first backward step points at the largest |1/d_i|); a matrix with an
    entrywise nonnegative inverse (the sign vector is all ones, so the
    backward step lands on the largest column sum);
  * in the factorization, the estimate only raises s_k = 1/est above the
    exact one, so it never turns an LU step of the exact criterion into QR.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

from paper_1401_5522_amd import inputs


def lapack_est(A):
    lu, _ = sla.lu_factor(A)
    anorm = np.abs(A).sum(axis=0).max()
    rcond, info = lapack.dgecon(lu, anorm, norm="1")
    assert info == 0
    return 1.0 / (rcond * anorm)


@pytest.mark.parametrize("m", [2, 3, 7, 32, 64, 255])
def test_estimate_equals_lapack_condition_estimator(O, m):
    rng = np.random.default_rng(500 + m)
    for t in range(6):
        A = rng.standard_normal((m, m)) * np.exp(rng.uniform(-3, 3, size=(1, m)))
        W, piv, z = O.gepp(A.copy())
        assert z == 0
        est = O.inv_norm1_est(W)
        ref = lapack_est(A)
        assert abs(est - ref) <= 1e-11 * ref, (m, t, est, ref)


@pytest.mark.parametrize("m", [1, 5, 40, 128])
def test_estimate_is_a_lower_bound(O, m):
    rng = np.random.default_rng(600 + m)
    for t in range(8):
        A = rng.standard_normal((m, m))
        if t % 2:  # ill-conditioned: one tiny singular value
            U, _, Vt = np.linalg.svd(A)
            sv = np.ones(m)
            sv[-1] = 1e-9
            A = (U * sv) @ Vt
        W, piv, _ = O.gepp(A.copy())
        est, exact = O.inv_norm1_est(W), O.inv_norm1(W, piv)
        assert est <= exact * (1 + 1e-12)


def test_estimate_exact_cases(O):
    # n = 1
    W, piv, _ = O.gepp(np.array([[-4.0]]))
    assert O.inv_norm1_est(W) == 0.25
    # diagonal
    d = np.array([3.0, -0.5, 8.0, 2.0, -0.25, 1.0])
    W, piv, _ = O.gepp(np.diag(d))
    assert O.inv_norm1_est(W) == 4.0 == O.inv_norm1(W, piv)
    # nonnegative inverse: lower bidiagonal, positive diagonal, negative subdiagonal
    m = 9
    A = np.diag(np.linspace(1.0, 3.0, m)) - np.diag(np.full(m - 1, 0.7), -1)
    assert (np.linalg.inv(A) >= 0).all()
    W, piv, _ = O.gepp(A.copy())
    exact = np.abs(np.linalg.inv(A)).sum(axis=0).max()
    assert abs(O.inv_norm1_est(W) - exact) <= 1e-14 * exact


def test_factor_with_estimate_only_raises_s(O):
    N, nb = 320, 32
    A = inputs.gaussian(N, seed=(610,))
    ex = O.factor(A, nb, "max", 40.0, forced=None)
    es = O.factor(A, nb, "max", 40.0, estimate=True)
    # while the decisions agree the factorizations are identical, so s can be compared
    k = 0
    while k < len(ex.dec) and ex.dec[k] == es.dec[k]:
        assert es.s[k] >= ex.s[k] * (1 - 1e-12), k
        np.testing.assert_array_equal(es.m[k], ex.m[k])
        k += 1
    if k < len(ex.dec):  # first difference: the estimate can only have turned QR into LU
        assert ex.dec[k] == 0 and es.dec[k] == 1
    assert 0 < ex.dec.sum() < len(ex.dec)
