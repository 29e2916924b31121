"""Pins of the oracle's diagonal-domain variant (Sec. 2.1, last paragraph;
Sec. 3.1: the criterion sees A_kk after the domain's interchanges; Sec. 3.3:
MUMPS's local and away maxima are over and off the domain).

What fixes the answer independently of the oracle:
  * a stride p >= n leaves the diagonal tile alone in every domain: the
    results equal the tile-only factorization bit for bit;
  * p = 1 puts the whole panel in the domain: with alpha = inf every step is
    an LU step with partial pivoting over the whole panel, i.e. LAPACK's
    blocked LU with partial pivoting (scipy lu_factor): same pivots, same U,
    and the same L once later interchanges are applied to earlier columns;
  * with p = 1 and a finite alpha, while every step so far was LU, the
    decision equals the Max test recomputed from the dense Schur complement
    with scipy's partial pivoting of its first block column;
  * MUMPS with p = 1 has no tile off the domain (away_max = 0): every step
    is an LU step, and the factorization is again LAPACK's;
  * every forced LU/QR sequence with p = 2 solves A x = b (brute force).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_5522_amd import inputs


def global_pivots(f, N, nb):
    """Row exchanged with global row k*nb + c at column c of each LU step."""
    n = (N + nb - 1) // nb
    out = np.zeros(N, dtype=np.int64)
    for k in range(n):
        mk = min(nb, N - k * nb)
        for c in range(mk):
            s = int(f.ipiv[k * nb + c])
            tiles = [k] + list(range(k + f.domain, n, f.domain)) if f.domain else [k]
            out[k * nb + c] = tiles[s // nb] * nb + s % nb
    return out


@pytest.mark.parametrize("crit,alpha", [("max", 300.0), ("sum", 40.0), ("mumps", 2.0)])
def test_stride_beyond_panel_is_the_tile_variant(O, crit, alpha):
    N, nb = 200, 16
    A = inputs.gaussian(N, seed=(60,))
    b = inputs.rhs(N, seed=(61,))
    t = O.factor(A, nb, crit, alpha)
    d = O.factor(A, nb, crit, alpha, domain=(N + nb - 1) // nb)
    np.testing.assert_array_equal(t.F, d.F)
    np.testing.assert_array_equal(t.dec, d.dec)
    np.testing.assert_array_equal(t.s, d.s)
    np.testing.assert_array_equal(t.m, d.m)
    np.testing.assert_array_equal(t.margin, d.margin)
    np.testing.assert_array_equal(t.solve(b), d.solve(b))


@pytest.mark.parametrize("N,nb", [(96, 16), (100, 16), (64, 8)])
def test_whole_panel_domain_at_inf_alpha_is_lapack_getrf(O, N, nb):
    A = inputs.gaussian(N, seed=(62, N))
    f = O.factor(A, nb, "max", np.inf, domain=1)
    assert (f.dec == 1).all()
    lu, piv = sla.lu_factor(A)
    gp = global_pivots(f, N, nb)
    np.testing.assert_array_equal(gp, piv)
    scale = np.abs(lu).max()
    U, Uo = np.triu(f.F), np.triu(lu)
    assert np.abs(U - Uo).max() <= 1e-13 * scale
    # L: the oracle applies step k's interchanges to the trailing columns only;
    # LAPACK applies every later interchange to the earlier columns as well
    L = np.tril(f.F, -1)
    for r in range(N):
        k = r // nb
        p = gp[r]
        if p != r:  # rows r and p swap in the columns left of step k
            L[[r, p], : k * nb] = L[[p, r], : k * nb]
    assert np.abs(L - np.tril(lu, -1)).max() <= 1e-13 * max(np.abs(np.tril(lu, -1)).max(), 1.0)
    b = inputs.rhs(N, seed=(63, N))
    np.testing.assert_allclose(f.solve(b), sla.lu_solve((lu, piv), b), rtol=1e-10, atol=0)


def dense_domain_decisions(A, nb, alpha):
    """Max decisions with the whole panel as the domain, from the dense Schur
    complement: the first block column is pivoted by scipy's LU, the
    diagonal tile after pivoting gives s, the permuted tiles below give m.
    Stops at the first QR step (the Schur complement is then no longer that
    of an LU factorization)."""
    S = np.array(A, dtype=np.float64)
    out = []
    while S.shape[0] > 0:
        m_k = min(nb, S.shape[0])
        P, _, _ = sla.lu(S[:, :m_k])
        Sp = P.T @ S                              # rows in pivoted order
        Akk = Sp[:m_k, :m_k]
        s = 1.0 / np.linalg.norm(np.linalg.inv(Akk), 1)
        m = 0.0
        for r0 in range(m_k, S.shape[0], nb):
            m = max(m, np.linalg.norm(Sp[r0:r0 + nb, :m_k], 1))
        lu = alpha * s >= m
        out.append((lu, s, m))
        if not lu:
            break
        S = Sp[m_k:, m_k:] - Sp[m_k:, :m_k] @ np.linalg.solve(Akk, Sp[:m_k, m_k:])
    return out


@pytest.mark.parametrize("alpha", [30.0, 100.0, 200.0])
def test_whole_panel_domain_decisions_match_dense_schur(O, alpha):
    N, nb = 128, 16
    A = inputs.gaussian(N, seed=(64,))
    f = O.factor(A, nb, "max", alpha, domain=1)
    ref = dense_domain_decisions(A, nb, alpha)
    for k, (lu, s, m) in enumerate(ref):
        if abs(alpha * s - m) > 1e-9 * max(alpha * s, m):
            assert f.dec[k] == lu, k
        assert abs(f.s[k] - s) <= 1e-9 * s
        assert abs(f.m[k] - m) <= 1e-10 * max(m, 1e-300)
    assert any(lu for lu, _, _ in ref)


def test_mumps_with_whole_panel_domain_has_no_away_part(O):
    N, nb = 96, 16
    A = inputs.gaussian(N, seed=(65,))
    f = O.factor(A, nb, "mumps", 1e-3, domain=1)
    assert (f.dec == 1).all()                     # est = 0 <= alpha pivot for every column
    assert (f.m == 0.0).all()
    lu, piv = sla.lu_factor(A)
    assert np.abs(np.triu(f.F) - np.triu(lu)).max() <= 1e-13 * np.abs(lu).max()


@pytest.mark.parametrize("N,nb", [(16, 4), (18, 4)])
def test_every_forced_sequence_solves_with_domain(O, N, nb):
    n = (N + nb - 1) // nb
    A = inputs.gaussian(N, seed=(66, N))
    B = inputs.rhs(N, 2, seed=(67,))
    X0 = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A)
    for seq in itertools.product([0, 1], repeat=n):
        f = O.factor(A, nb, "forced", forced=np.array(seq, dtype=np.int8), domain=2)
        X = f.solve(B)
        assert np.abs(X - X0).max() <= kappa * 1e-13 * np.abs(X0).max(), seq


def test_domain_raises_lu_fraction_on_random_matrices(O):
    # Sec. 5: factoring the diagonal domain makes an LU step more likely
    N, nb = 256, 16
    A = inputs.gaussian(N, seed=(68,))
    tile = O.factor(A, nb, "max", 100.0)
    dom = O.factor(A, nb, "max", 100.0, domain=1)
    assert dom.dec.sum() > tile.dec.sum()


def test_augmented_and_second_pass_agree_with_domain(O):
    N, nb = 90, 8
    A = inputs.gaussian(N, seed=(69,))
    b = inputs.rhs(N, seed=(70,))
    f = O.factor(A, nb, "max", 50.0, domain=3, B=b)
    y = O.forward(f, b)[:, 0]
    np.testing.assert_allclose(f.Bt[:, 0], y, rtol=1e-13, atol=1e-13 * np.abs(y).max())
    assert 0 < f.dec.sum() < len(f.dec)
