"""Pins of the oracle's QR elimination trees (Sec. 2.2, Alg. 3 with the TS
kernels of Alg. 4a inside groups of S tiles and the TT kernels of Alg. 4b
over the groups' heads, binary).

What fixes the answer independently of the oracle's tree code:
  * TTQRT/TTMQR are TSQRT/TSMQR on a triangular bottom tile with the zero
    products left out: bitwise equal, tails upper triangular, and the
    reflectors orthogonal ([R1; R2] = Q [R; 0] with Q^T Q = I);
  * whatever the tree, one QR step leaves R_kk and the rows of tile row k
    equal to LAPACK's QR of the block column up to the sign of each row, and
    the trailing block below row k differs between trees by an orthogonal
    transformation of its rows, so its Gram matrix is tree-invariant (and
    equals A^T A - R_k^T R_k);
  * S >= n - k is the flat tree (bitwise), and every forced sequence with a
    tree solves A x = b (brute force, ragged last tile included);
  * the elimination structure: exactly the killed heads hold TT factors.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla


def _tri(rng, m):
    return np.triu(rng.standard_normal((m, m)))


@pytest.mark.parametrize("m", [1, 3, 8, 16])
def test_ttqrt_is_tsqrt_on_triangular_tiles(O, m):
    rng = np.random.default_rng(950 + m)
    R1, R2 = _tri(rng, m), _tri(rng, m)
    a1, a2, Ta = O.ttqrt(R1.copy(), R2.copy())
    b1, b2, Tb = O.tsqrt(R1.copy(), R2.copy())
    assert np.array_equal(a1, b1) and np.array_equal(Ta, Tb)
    assert np.array_equal(np.triu(a2), np.triu(b2))
    assert np.array_equal(np.tril(b2, -1), np.zeros((m, m)))  # TS keeps the zeros exactly
    C1, C2 = rng.standard_normal((m, 5)), rng.standard_normal((m, 5))
    x1, x2 = O.ttmqr(np.triu(a2), Ta, C1.copy(), C2.copy())
    y1, y2 = O.tsmqr(np.triu(b2), Tb, C1.copy(), C2.copy())
    assert np.array_equal(x1, y1) and np.array_equal(x2, y2)


def test_tt_reflectors_are_orthogonal(O):
    rng = np.random.default_rng(960)
    m = 12
    R1, R2 = _tri(rng, m), _tri(rng, m)
    r1, y, T = O.ttqrt(R1.copy(), R2.copy())
    Qt1, Qt2 = O.ttmqr(np.triu(y), T, np.eye(2 * m)[:m].copy(), np.eye(2 * m)[m:].copy())
    Qt = np.vstack([Qt1, Qt2])
    assert np.allclose(Qt @ Qt.T, np.eye(2 * m), atol=1e-13)
    top, bot = O.ttmqr(np.triu(y), T, R1.copy(), R2.copy())
    assert np.allclose(top, np.triu(r1), atol=1e-13) and np.allclose(bot, 0, atol=1e-13)


@pytest.mark.parametrize("S", [1, 2, 3])
def test_tree_qr_step_matches_lapack_and_gram(O, S):
    rng = np.random.default_rng(970 + S)
    N, nb = 112, 16  # seven tiles
    A = rng.standard_normal((N, N))
    seq = np.zeros(7, np.int8)
    f = O.factor(A, nb, "forced", forced=seq, nsteps=1, tree=S)
    flat = O.factor(A, nb, "forced", forced=seq, nsteps=1, tree=0)
    Q, R = sla.qr(A[:, :nb])
    Rk = np.hstack([R[:nb], (Q.T @ A[:, nb:])[:nb]])
    got = np.hstack([np.triu(f.F[:nb, :nb]), f.F[:nb, nb:]])
    assert np.allclose(np.abs(got), np.abs(Rk), atol=1e-11 * np.abs(Rk).max())
    T2 = f.F[nb:, nb:]
    G = A[:, nb:].T @ A[:, nb:] - Rk[:, nb:].T @ Rk[:, nb:]
    assert np.allclose(T2.T @ T2, G, atol=1e-10 * np.abs(G).max())
    F2 = flat.F[nb:, nb:]
    assert np.allclose(T2.T @ T2, F2.T @ F2, atol=1e-10 * np.abs(G).max())
    assert not np.allclose(T2, F2)  # a different tree: a different basis of the trailing rows


def test_large_group_is_the_flat_tree(O):
    rng = np.random.default_rng(980)
    N, nb = 90, 16
    A = rng.standard_normal((N, N))
    b = rng.standard_normal(N)
    f0 = O.factor(A, nb, "max", 1.0)
    f9 = O.factor(A, nb, "max", 1.0, tree=9)
    assert np.array_equal(f0.F, f9.F) and np.array_equal(f0.dec, f9.dec)
    assert np.array_equal(f0.solve(b), f9.solve(b))
    assert not f9.Tt.any()


@pytest.mark.parametrize("S,N,nb", [(1, 40, 8), (2, 37, 8), (3, 48, 8)])
def test_tree_every_forced_sequence_solves(O, S, N, nb):
    rng = np.random.default_rng(990 + S)
    A = rng.standard_normal((N, N))
    b = rng.standard_normal(N)
    xref = np.linalg.solve(A, b)
    n = (N + nb - 1) // nb
    for seq in itertools.product([0, 1], repeat=n):
        f = O.factor(A, nb, "forced", forced=np.array(seq, np.int8), tree=S)
        x = f.solve(b)
        assert np.linalg.norm(x - xref) <= 1e-10 * np.linalg.norm(xref), seq


def test_tree_augmented_rhs_matches_forward_replay(O):
    rng = np.random.default_rng(995)
    N, nb = 96, 16
    A = rng.standard_normal((N, N))
    B = rng.standard_normal((N, 2))
    f = O.factor(A, nb, "forced", forced=np.array([0, 1, 0, 0, 1, 0], np.int8), B=B, tree=2)
    Y = O.forward(f, B)
    assert np.allclose(f.Bt, Y, rtol=0, atol=1e-12 * np.abs(Y).max())


def test_tree_structure(O):
    """Step 0 of seven tiles with S = 2: groups {0,1}, {2,3}, {4,5,6} (a last
    group of one tile joins the one before), heads 0, 2, 4; the binary tree
    kills head 2 by 0 (d = 1) and head 4 by 0 (d = 2).  Step 1 (six tiles):
    groups {1,2}, {3,4}, {5,6}, heads 1, 3, 5: 3 killed by 1, 5 by 1."""
    rng = np.random.default_rng(996)
    N, nb = 112, 16
    n = 7
    A = rng.standard_normal((N, N))
    f = O.factor(A, nb, "forced", forced=np.zeros(n, np.int8), nsteps=2, tree=2)
    Tt = f.Tt.reshape(n, n, nb * nb)  # [k][i]
    killed = {k: sorted(i for i in range(n) if Tt[k, i].any()) for k in range(2)}
    assert killed == {0: [2, 4], 1: [3, 5]}
    Tq = f.Tq.reshape(n, n, nb * nb)
    assert all(Tq[0, i].any() for i in range(n)) and not Tq[0, :0].any()
