"""Pins of the oracle's tile routines against library routines and closed forms.

Each test compares a routine of the oracle with something other than itself:
LAPACK through scipy (GETRF pivots and factors, GEQRF reflectors and tau),
numpy (inverse, norms, QR), or an exact mathematical identity.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_5522_amd import inputs

U = 2.0 ** -53


@pytest.mark.parametrize("m", [1, 2, 5, 32, 64])
def test_gepp_equals_lapack_getrf(O, m):
    A = inputs.gaussian(m, seed=(11,))
    W, ipiv, z = O.gepp(A)
    lu, piv = sla.lu_factor(A)
    assert z == 0
    np.testing.assert_array_equal(ipiv, piv)
    np.testing.assert_allclose(W, lu, rtol=0, atol=1e-13 * np.abs(lu).max())


def test_gepp_no_interchange_on_column_diagonally_dominant(O):
    # Gaussian elimination with partial pivoting makes no interchange on a
    # matrix diagonally dominant by columns (Wilkinson; Higham ASNA ch. 9).
    G = inputs.gaussian(48, seed=(12,))
    A = G + np.diag(np.abs(G).sum(axis=0) + 1.0)
    assert np.all(2 * np.abs(np.diag(A)) > np.abs(A).sum(axis=0))
    _, ipiv, _ = O.gepp(A)
    np.testing.assert_array_equal(ipiv, np.arange(48))


def test_gepp_first_max_tie_break_and_zero_column(O):
    A = np.array([[1.0, 2.0, 0.0], [-1.0, 1.0, 0.0], [1.0, 0.0, 0.0]])
    W, ipiv, z = O.gepp(A)
    assert ipiv[0] == 0          # |1| = |-1| = |1|: the first row wins
    assert z == 3                # third column is exactly zero
    assert ipiv[2] == 2


@pytest.mark.parametrize("m", [1, 7, 32])
def test_inverse_norm_matches_numpy(O, m):
    A = inputs.gaussian(m, seed=(13,)) + 3 * np.eye(m)
    W, ipiv, _ = O.gepp(A)
    got = O.inv_norm1(W, ipiv)
    ref = np.linalg.norm(np.linalg.inv(A), 1)
    assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("alpha", [1.0, 2.0, 4.0, 0.5])
def test_inverse_norm_exact_on_scaled_identity(O, alpha):
    A = np.eye(16) / alpha
    W, ipiv, _ = O.gepp(A)
    assert O.inv_norm1(W, ipiv) == alpha


def test_inverse_norm_invariant_under_row_permutation(O):
    # ||(PA)^{-1}||_1 = ||A^{-1} P^T||_1 = ||A^{-1}||_1: a column permutation
    # leaves the 1-norm unchanged, so factoring before or after pivoting does
    # not change the criterion.
    A = inputs.gaussian(24, seed=(14,))
    P = np.random.default_rng(0).permutation(24)
    a = O.inv_norm1(*O.gepp(A)[:2])
    b = O.inv_norm1(*O.gepp(A[P])[:2])
    assert abs(a - b) <= 1e-12 * a


def test_tile_norm1_matches_numpy(O):
    A = inputs.gaussian(20, seed=(15,))[:, :13]
    assert abs(O.tile_norm1(A) - np.linalg.norm(A, 1)) <= 1e-14 * np.linalg.norm(A, 1)


def _house_product(V, tau):
    m = V.shape[0]
    Q = np.eye(m)
    for c in range(len(tau)):
        v = np.zeros(m)
        v[c] = 1.0
        v[c + 1:] = V[c + 1:, c]
        Q = Q @ (np.eye(m) - tau[c] * np.outer(v, v))
    return Q


@pytest.mark.parametrize("m", [1, 2, 9, 32])
def test_geqrt_equals_lapack_geqrf(O, m):
    A = inputs.gaussian(m, seed=(16,))
    F, T = O.geqrt(A)
    (h, tau), _ = sla.qr(A, mode="raw")
    np.testing.assert_allclose(np.triu(F), np.triu(h), atol=1e-13 * np.abs(A).max() * m)
    np.testing.assert_allclose(np.tril(F, -1), np.tril(h, -1), atol=1e-13 * m)
    np.testing.assert_allclose(np.diag(T), tau, atol=1e-14)
    # compact WY: I - V T V^T equals the product of the elementary reflectors
    V = np.tril(F, -1) + np.eye(m)
    np.testing.assert_allclose(np.eye(m) - V @ T @ V.T, _house_product(F, tau), atol=1e-13 * m)


def test_geqrt_zero_tail_gives_identity_reflector(O):
    A = np.triu(inputs.gaussian(6, seed=(17,)))
    F, T = O.geqrt(A)
    np.testing.assert_array_equal(F, A)           # already triangular: tau = 0, nothing changes
    np.testing.assert_array_equal(T, np.zeros((6, 6)))


def test_unmqr_applies_q_transpose(O):
    A = inputs.gaussian(12, seed=(18,))
    C = inputs.gaussian(12, seed=(19,))[:, :7]
    F, T = O.geqrt(A)
    V = np.tril(F, -1) + np.eye(12)
    Q = np.eye(12) - V @ T @ V.T
    np.testing.assert_allclose(O.unmqr(F, T, C), Q.T @ C, atol=1e-13 * 12)
    np.testing.assert_allclose(Q.T @ A, np.triu(F), atol=1e-12)


@pytest.mark.parametrize("mk,mi", [(8, 8), (8, 3), (1, 5), (16, 16)])
def test_tsqrt_tsmqr_against_explicit_q(O, mk, mi):
    R0 = np.triu(inputs.gaussian(mk, seed=(20,)))
    A0 = inputs.gaussian(max(mi, mk), seed=(21,))[:mi, :mk]
    R, Y, T = O.tsqrt(R0, A0)
    V = np.vstack([np.eye(mk), Y])
    Q = np.eye(mk + mi) - V @ T @ V.T
    stacked = np.vstack([R0, A0])
    np.testing.assert_allclose(Q.T @ Q, np.eye(mk + mi), atol=1e-13 * (mk + mi))
    np.testing.assert_allclose(Q.T @ stacked, np.vstack([np.triu(R), np.zeros((mi, mk))]),
                               atol=1e-12 * np.abs(stacked).max())
    # R is unique up to row signs (full rank): compare magnitudes with numpy's QR
    Rn = np.linalg.qr(stacked, mode="r")
    np.testing.assert_allclose(np.abs(np.triu(R)), np.abs(Rn), atol=1e-12 * np.abs(stacked).max())
    Ck = inputs.gaussian(max(mk, 5), seed=(22,))[:mk, :5]
    Ci = inputs.gaussian(max(mi, 5), seed=(23,))[:mi, :5]
    Ck2, Ci2 = O.tsmqr(Y, T, Ck, Ci)
    ref = Q.T @ np.vstack([Ck, Ci])
    np.testing.assert_allclose(np.vstack([Ck2, Ci2]), ref, atol=1e-13 * (mk + mi) * 4)


def test_splitmix64_published_vector(O):
    # SplitMix64 seeded with 1234567: the first outputs of the published
    # generator (Steele, Lea, Flood 2014; Vigna's reference implementation).
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [O.splitmix64(1234567, k) for k in range(5)] == want
    u = O.uniform(1234567, 0)
    assert u == (6457827717110365317 >> 11) * 2.0 ** -53
