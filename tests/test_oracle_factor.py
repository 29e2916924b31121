"""Pins of the oracle's whole factorization and solve.

What fixes the answer here, independently of the oracle itself:
  * the worked growth example of Sec. 3.1 lifted to tiles (exact ties, exact
    final tile (1+alpha)^(n-1) I, growth bound attained);
  * the extreme thresholds alpha = 0 (tiled QR: orthogonal Q, |R| of numpy's
    QR) and alpha = inf / diagonal dominance (block LU without pivoting equals
    the unpivoted scalar LU);
  * block diagonal dominance => every Max and Sum test passes (Sec. 3.2);
  * decisions recomputed from dense Schur complements while all steps so far
    were LU (the Schur complement does not depend on how A_kk is factored);
  * brute-force dense solves for every forced LU/QR sequence on tiny inputs;
  * the per-step growth inequalities and growth bounds of Sec. 3.1 and 3.2;
  * the Table 1 flop totals (exactly 2N^3/3 and 4N^3/3).
"""
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_5522_amd import inputs

U = 2.0 ** -53


def tiles(N, nb):
    return (N + nb - 1) // nb


# ---------------------------------------------------------------- worked example
@pytest.mark.parametrize("alpha,n,nb", [(1.0, 6, 4), (2.0, 5, 3), (4.0, 4, 2), (1.0, 10, 1), (2.0, 8, 2)])
def test_kron_worked_example_exact_ties_and_growth(O, alpha, n, nb):
    A = inputs.kron_example(n, nb, alpha)
    f = O.factor(A, nb, "max", alpha)
    assert f.dec.tolist() == [1] * n                      # alpha s = m exactly: ">=" takes LU
    np.testing.assert_array_equal(f.s[:-1], np.full(n - 1, 1.0 / alpha))
    assert f.s[-1] == (1 + alpha) ** (n - 1)               # the last tile is (1+alpha)^(n-1) I
    np.testing.assert_array_equal(f.m[:-1], np.ones(n - 1))
    assert f.m[-1] == 0.0                                  # empty sub-panel at the last step
    np.testing.assert_array_equal(f.margin[:-1], np.zeros(n - 1))
    assert f.margin[-1] == 1.0
    last = f.F[(n - 1) * nb:, (n - 1) * nb:]
    np.testing.assert_array_equal(np.triu(last), (1 + alpha) ** (n - 1) * np.eye(nb))
    # growth over tiles attains the bound (1+alpha)^(n-1) of Sec. 3.1 exactly
    assert f.diag[O.DG_GROWTH_TILE] == (1 + alpha) ** (n - 1) / max(1.0, 1.0 / alpha)


def test_kron_example_just_below_threshold_goes_qr(O):
    A = inputs.kron_example(4, 3, 2.0)
    f = O.factor(A, 3, "max", np.nextafter(2.0, 0.0))
    assert f.dec[0] == 0


# ---------------------------------------------------------------- extremes
@pytest.mark.parametrize("N,nb", [(37, 8), (64, 16), (20, 20)])
def test_alpha_zero_is_tiled_qr(O, N, nb):
    A = inputs.gaussian(N, seed=(30,))
    f = O.factor(A, nb, "max", 0.0)
    assert f.dec.tolist() == [0] * tiles(N, nb)
    Qt = O.forward(f, np.eye(N))                            # replaying on I gives Q^T
    assert np.linalg.norm(Qt @ Qt.T - np.eye(N)) <= 10 * N * U
    R = np.triu(f.F)
    Rn = np.linalg.qr(A, mode="r")
    np.testing.assert_allclose(np.abs(R), np.abs(Rn), atol=1e-12 * np.abs(A).max() * np.sqrt(N))
    np.testing.assert_allclose(Qt @ A, R, atol=1e-12 * np.abs(A).max() * np.sqrt(N))
    b = inputs.rhs(N, seed=(31,))
    x = f.solve(b)
    assert O.backward_error(A, x, b) <= N * U


@pytest.mark.parametrize("N,nb", [(40, 8), (45, 8), (64, 32)])
def test_all_lu_on_diagonally_dominant_is_unpivoted_lu(O, N, nb):
    G = inputs.gaussian(N, seed=(32,))
    A = G + np.diag(np.abs(G).sum(axis=0) + 1.0)          # strictly column diagonally dominant
    for crit, alpha in [("max", np.inf), ("sum", np.inf), ("mumps", np.inf)]:
        f = O.factor(A, nb, crit, alpha)
        assert f.dec.tolist() == [1] * tiles(N, nb)
        P, L, Uf = sla.lu(A)
        np.testing.assert_array_equal(P, np.eye(N))
        np.testing.assert_allclose(np.tril(f.F, -1) + np.eye(N), L, atol=1e-13)
        np.testing.assert_allclose(np.triu(f.F), Uf, atol=1e-13 * np.abs(A).max())
        np.testing.assert_array_equal(f.ipiv, np.concatenate([np.arange(min(nb, N - k)) for k in range(0, N, nb)]))


def test_block_diagonally_dominant_passes_every_test(O):
    # Sec. 3.2: for alpha >= 1 both criteria hold at every step when A is block
    # diagonally dominant by columns in the 1-norm.
    N, nb = 48, 8
    G = inputs.gaussian(N, seed=(33,))
    A = G.copy()
    n = N // nb
    for j in range(n):
        off = sum(np.linalg.norm(G[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb], 1) for i in range(n) if i != j)
        d = off + np.linalg.norm(G[j * nb:(j + 1) * nb, j * nb:(j + 1) * nb], 1) + 1.0
        A[j * nb:(j + 1) * nb, j * nb:(j + 1) * nb] += d * np.eye(nb)
    for j in range(n):
        Ajj = A[j * nb:(j + 1) * nb, j * nb:(j + 1) * nb]
        off = sum(np.linalg.norm(A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb], 1) for i in range(n) if i != j)
        assert 1.0 / np.linalg.norm(np.linalg.inv(Ajj), 1) >= off
    for crit in ("max", "sum"):
        f = O.factor(A, nb, crit, 1.0)
        assert f.dec.tolist() == [1] * n


# ---------------------------------------------------------------- decisions from Schur complements
def _dense_decisions(A, nb, crit, alpha):
    """Decisions, s_k and m_k from dense formulas while every earlier step is LU."""
    N = A.shape[0]
    n = tiles(N, nb)
    S = A.copy()
    out = []
    for k in range(n):
        o = k * nb
        mk = min(nb, N - o)
        Akk = S[o:o + mk, o:o + mk]
        s = 1.0 / np.linalg.norm(np.linalg.inv(Akk), 1)
        norms = [np.linalg.norm(S[i:i + nb, o:o + mk], 1) for i in range(o + mk, N, nb)]
        m = (max(norms) if crit == "max" else sum(norms)) if norms else 0.0
        lu = alpha * s >= m
        out.append((int(lu), s, m))
        if not lu:
            break
        # Schur complement of the leading block (independent of how A_kk is factored)
        B = S[o + mk:, o:o + mk]
        Cb = S[o:o + mk, o + mk:]
        S[o + mk:, o + mk:] -= B @ np.linalg.solve(Akk, Cb)
    return out


@pytest.mark.parametrize("crit,alpha,shift", [("max", 1.0, 3.0), ("max", 2.0, 1.5), ("sum", 1.0, 6.0),
                                              ("max", 0.5, 6.0), ("sum", 4.0, 1.0), ("max", 300.0, 0.0)])
@pytest.mark.parametrize("N,nb", [(48, 8), (50, 6), (24, 1)])
def test_decisions_match_dense_schur_complements(O, crit, alpha, shift, N, nb):
    A = inputs.gaussian(N, seed=(34, N)) + shift * np.sqrt(N) * np.eye(N)
    f = O.factor(A, nb, crit, alpha)
    ref = _dense_decisions(A, nb, crit, alpha)
    for k, (lu, s, m) in enumerate(ref):
        if abs(alpha * s - m) > 1e-9 * max(alpha * s, m):       # outside the rounding band
            assert f.dec[k] == lu, k
        assert abs(f.s[k] - s) <= 1e-10 * s
        assert abs(f.m[k] - m) <= 1e-10 * max(m, 1e-300)


def test_nb1_mumps_equals_max(O):
    # With 1x1 tiles the pivot is the tile, gf = 1, est = away_max: MUMPS is the
    # scalar threshold test alpha |a_kk| >= max_{i>k} |a_ik|, i.e. Max.
    A = inputs.gaussian(30, seed=(35,)) + 2.0 * np.eye(30)
    for alpha in (0.5, 1.0, 2.0):
        a = O.factor(A, 1, "max", alpha)
        b = O.factor(A, 1, "mumps", alpha)
        np.testing.assert_array_equal(a.dec, b.dec)
        np.testing.assert_array_equal(a.F, b.F)


def test_mumps_zero_away_part_is_lu(O):
    N, nb = 24, 8
    A = np.triu(inputs.gaussian(N, seed=(36,))) + 4 * np.eye(N)
    f = O.factor(A, nb, "mumps", 1.0)
    assert f.dec.tolist() == [1, 1, 1]


# Hand computation for inputs.mumps_example (Sec. 3.3, eq. mumps), step 0:
#   GEPP on A_00's leading block [[4,2,2],[2,5,3],[0,2,4]]: column 0 pivots on
#   4 (row 0), multipliers 1/2 and 0, rows 1, 2 become [4, 2] and [2, 4];
#   column 1 pivots on 4 (row 1), multiplier 1/2, and the last entry becomes
#   4 - 2/2 = 3.  No interchanges; pivot = (4, 4, 3) (8 on the rest).
#   local_max = (4, 5, 4), so growth_factor = (1, 4/5, 3/4) (1 on the rest).
#   away_max = (1, 4, 5) (0 on the rest).
# The estimate starts at away_max(j) and step i of the GEPP multiplies it by
# growth_factor(i).  Three readings of which columns step i touches:
#   chosen, i < j (the columns step i has not yet pivoted): est = (1, 4, 4)
#   (a) only i = j:                                         est = (1, 3.2, 3.75)
#   (b) every i:                    est = 0.6 away_max =          (0.6, 2.4, 3)
# LU iff alpha pivot(j) >= est(j) for all j, i.e. alpha >= max_j est/pivot:
#   chosen 4/3, (a) 1.25, (b) 1.
# The margin is min_j (alpha pivot(j) - est(j)) / max(alpha pivot(j), est(j)).
MUMPS_HAND = {
    # reading: (m = max est, [(alpha, decision, margin)])
    0: (4.0, [(1.3, 0, (3.9 - 4.0) / 4.0), (1.4, 1, (4.2 - 4.0) / 4.2)]),
    1: (3.75, [(1.3, 1, (3.9 - 3.75) / 3.9), (1.2, 0, (3.6 - 3.75) / 3.75)]),
    2: (3.0, [(1.3, 1, (3.9 - 3.0) / 3.9), (0.9, 0, (2.7 - 3.0) / 3.0)]),
}


@pytest.mark.parametrize("nb", [3, 5])
def test_mumps_estimate_hand_example(O, nb):
    A = inputs.mumps_example(nb)
    for reading, (m, cases) in MUMPS_HAND.items():
        for alpha, lu, margin in cases:
            f = O.factor(A, nb, "mumps", alpha, mumps_reading=reading)
            assert f.dec[0] == lu, (reading, alpha)
            assert f.s[0] == 3.0                       # smallest pivot
            assert f.m[0] == pytest.approx(m, rel=1e-15, abs=0), (reading, alpha)
            assert f.margin[0] == pytest.approx(margin, rel=1e-13), (reading, alpha)
    # at alpha = 1.3 the chosen reading takes QR while both rejected readings take LU
    assert [O.factor(A, nb, "mumps", 1.3, mumps_reading=r).dec[0] for r in (0, 1, 2)] == [0, 1, 1]


# ---------------------------------------------------------------- solve
@pytest.mark.parametrize("N,nb", [(12, 4), (14, 4), (9, 3), (16, 4)])
def test_every_forced_sequence_solves(O, N, nb):
    n = tiles(N, nb)
    A = inputs.gaussian(N, seed=(37, N)) + 0.5 * np.sqrt(N) * np.eye(N)
    B = inputs.rhs(N, 3, seed=(38,))
    X0 = np.linalg.solve(A, B)
    kappa = np.linalg.cond(A)
    for seq in itertools.product([0, 1], repeat=n):
        f = O.factor(A, nb, "forced", forced=np.array(seq, dtype=np.int8))
        assert f.dec.tolist() == list(seq)
        X = f.solve(B)
        assert np.linalg.norm(X - X0) <= 1e-12 * kappa * np.linalg.norm(X0), seq


@pytest.mark.parametrize("crit,alpha", [("max", 1.0), ("random", 50.0), ("max", np.inf), ("sum", 2.0)])
def test_augmented_equals_second_pass(O, crit, alpha):
    # Sec. 2.4: transforming [A, b] during the factorization and replaying the
    # stored transforms afterwards are the same operations on b.
    N, nb = 45, 8
    A = inputs.gaussian(N, seed=(39,)) + 2 * np.eye(N)
    B = inputs.rhs(N, 2, seed=(40,))
    f = O.factor(A, nb, crit, alpha, seed=5, B=B)
    Y = O.forward(f, B)
    np.testing.assert_array_equal(f.Bt, Y)
    x = O.backward(f, f.Bt)
    np.testing.assert_array_equal(x, f.solve(B))


def test_random_choice_frequency(O):
    N = 600
    A = inputs.gaussian(N, seed=(41,)) + 40 * np.eye(N)
    for alpha in (10.0, 50.0, 90.0):
        f = O.factor(A, 1, "random", alpha, seed=123)
        frac = f.dec.mean()
        sd = np.sqrt(alpha / 100 * (1 - alpha / 100) / N)
        assert abs(frac - alpha / 100) <= 4 * sd
        u = np.array([O.uniform(123, k) for k in range(N)])
        np.testing.assert_array_equal(f.dec, (u < alpha / 100).astype(np.int8))


# ---------------------------------------------------------------- growth bounds
@pytest.mark.parametrize("alpha", [0.5, 1.0, 4.0, 16.0])
@pytest.mark.parametrize("kind", ["gaussian", "diag_dominant", "growth_prone"])
def test_max_criterion_step_inequality(O, alpha, kind):
    N, nb = 64, 8
    A = inputs.matrix(kind, N, seed=(42,)) + (0 if kind != "gaussian" else 3.0 * np.sqrt(N) * np.eye(N))
    f = O.factor(A, nb, "max", alpha)
    n = tiles(N, nb)
    slack = 1 + 4 * nb * U * 10
    assert f.diag[O.DG_MAXINEQ] <= slack
    if f.dec.all():
        assert f.diag[O.DG_GROWTH_TILE] <= (1 + alpha) ** (n - 1) * slack


@pytest.mark.parametrize("kind", ["gaussian", "diag_dominant"])
def test_sum_criterion_step_inequality_and_linear_growth(O, kind):
    N, nb = 64, 8
    A = inputs.matrix(kind, N, seed=(43,)) + (0 if kind != "gaussian" else 6.0 * np.sqrt(N) * np.eye(N))
    f = O.factor(A, nb, "sum", 1.0)
    slack = 1 + 4 * nb * U * 10
    assert f.diag[O.DG_SUMINEQ] <= slack
    assert f.diag[O.DG_MAXINEQ] <= slack
    if f.dec.all():
        assert f.diag[O.DG_GROWTH_TILE] <= tiles(N, nb) * slack


def test_elementwise_growth_at_most_two_on_column_diagonally_dominant(O):
    G = inputs.gaussian(64, seed=(44,))
    A = G + np.diag(np.abs(G).sum(axis=0) + 1.0)
    f = O.factor(A, 8, "max", np.inf)
    assert f.diag[O.DG_GROWTH_ELEM] <= 2.0


# ---------------------------------------------------------------- flops, edge cases
@pytest.mark.parametrize("n,nb", [(1, 4), (5, 3), (16, 8)])
def test_table1_totals(O, n, nb):
    N = n * nb
    assert abs(O.true_flops(N, nb, np.ones(n, np.int8)) - 2 * N ** 3 / 3) <= 1e-9 * N ** 3
    assert abs(O.true_flops(N, nb, np.zeros(n, np.int8)) - 4 * N ** 3 / 3) <= 1e-9 * N ** 3


def test_singular_diagonal_tile_goes_qr_and_inf_alpha_sets_info(O):
    N, nb = 24, 8
    A = inputs.gaussian(N, seed=(45,))
    A[:8, :8] = 0.0
    f = O.factor(A, nb, "max", 1e30)
    assert f.dec[0] == 0 and f.s[0] == 0.0
    b = inputs.rhs(N, seed=(46,))
    assert O.backward_error(A, f.solve(b), b) <= N * U * 10
    g = O.factor(A, nb, "max", np.inf)
    assert g.dec[0] == 1 and g.diag[O.DG_INFO] == 1.0


def test_nan_input_goes_qr_and_flags(O):
    N, nb = 24, 8
    A = inputs.gaussian(N, seed=(47,)) + 10 * np.eye(N)
    A[20, 2] = np.nan
    f = O.factor(A, nb, "max", 1.0)
    assert f.dec[0] == 0 and f.diag[O.DG_NONFINITE] == 1.0


def test_single_tile_and_n_smaller_than_nb(O):
    for N in (1, 5):
        A = inputs.gaussian(N, seed=(48,)) + 3 * np.eye(N)
        b = inputs.rhs(N, seed=(49,))
        f = O.factor(A, 8, "max", 1.0)
        assert f.dec.tolist() == [1]
        np.testing.assert_allclose(f.solve(b), np.linalg.solve(A, b), rtol=1e-12)


def test_thread_count_invariance(O, tmp_path):
    code = r"""
import sys, numpy as np
sys.path.insert(0, %r)
from oracle import oracle as O
from paper_1401_5522_amd import inputs
A = inputs.gaussian(96, seed=(50,))
f = O.factor(A, 16, "max", 3000.0)
np.save(sys.argv[1], np.concatenate([f.F.ravel(order='F'), f.Tq, f.dec.astype(float)]))
""" % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "5"):
        p = tmp_path / f"o{t}.npy"
        env = dict(os.environ, OMP_NUM_THREADS=t)
        subprocess.check_call([sys.executable, "-c", code, str(p)], env=env)
        outs.append(np.load(p))
    np.testing.assert_array_equal(outs[0], outs[1])
