/*
 * Plain FP64 CPU oracle of the hybrid tiled LU-QR factorization and solve
 * (Faverge, Herrmann, Langou, Lowery, Robert, Dongarra, "Designing LU-QR
 * hybrid solvers for performance and stability", arXiv 1401.5522).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Everything is written as plain loops in the order the paper states the
 * method; OpenMP is used only to run independent tiles of one step side by
 * side (every tile is computed by exactly one thread, in a fixed order, so
 * results do not depend on the thread count).
 *
 * Storage conventions (all column-major):
 *   A      N x N, leading dimension lda.  Tile (i,j), 0-based, starts at
 *          A[i*nb + j*nb*lda]; tile sizes are nb except the last, which has
 *          N - (n-1)*nb rows/columns (the clean-up case of Sec. 2.4).
 *   On exit A holds, per step k:
 *     LU step: L\U of the diagonal tile, L_ik = A_ik U_kk^{-1} below it,
 *              U_kj = L_kk^{-1} P_kk A_kj to its right (Alg. 2).
 *     QR step: V\R of the diagonal tile (unit lower V), the TS reflector
 *              tails Y_ik below it, Q^T A_kj to its right (Alg. 3/4a).
 *     LU step, variant A2 (lu_variant = 2, Sec. 2.3): V\U of the GEQRT of
 *              the diagonal tile, L_ik = A_ik U_kk^{-1} below it,
 *              U_kj = Q_kk^T A_kj to its right; ipiv is the identity and
 *              Tq(k,k) holds the GEQRT factor.
 *   Tq     n*n blocks of nb*nb: block (i,k) at Tq + (k*n + i)*nb*nb holds the
 *          upper-triangular compact-WY factor of the reflectors that
 *          eliminated tile (i,k) (TSQRT), or of GEQRT for i == k.
 *   With an elimination tree (qr_tree = S > 0, oracle_factor_t): the
 *          heads of the groups of S tiles keep the unit-lower V of their
 *          GEQRT below the diagonal and Tq(h,k) holds its factor; a head h
 *          later killed by another head keeps the TTQRT reflector tails
 *          (upper triangular) on and above its diagonal, and Tt(h,k) (same
 *          layout as Tq) holds their factor.
 *   ipiv   N ints: for an LU step k, ipiv[k*nb + c] is the local row (0-based
 *          within tile k) exchanged with local row c at column c of GETRF.
 *          QR steps store the identity.
 *   dec    n bytes: 1 = LU step, 0 = QR step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

enum { CRIT_MAX = 0, CRIT_SUM = 1, CRIT_MUMPS = 2, CRIT_RANDOM = 3, CRIT_FORCED = 4 };

/* Diagnostics vector layout (oracle_factor's diag argument). */
enum {
    DG_INFO = 0,        /* first exactly-zero pivot of an LU step, 1-based global row; 0 if none */
    DG_NONFINITE = 1,   /* 1 if a criterion input was NaN/Inf */
    DG_GROWTH_TILE = 2, /* max_k max_{i,j>=k} ||A_ij^(k)||_1 / max_{i,j} ||A_ij||_1 */
    DG_GROWTH_ELEM = 3, /* same with max |a| elementwise */
    DG_MAXINEQ = 4,     /* max over LU steps, i,j>k of ||A_ij^(k+1)|| / (||A_ij^(k)|| + a||A_kj^(k)||) */
    DG_SUMINEQ = 5,     /* max over LU steps, j>k of the column-sum analogue (Sum criterion) */
    DG_TRUEFLOPS = 6,   /* Table 1 flop count of the steps taken (units of flops) */
    DG_NLU = 7,         /* number of LU steps */
    DG_COUNT = 8
};

static int64_t tsize(int64_t N, int64_t nb, int64_t i)
{
    int64_t n = (N + nb - 1) / nb;
    return (i < n - 1) ? nb : N - (n - 1) * nb;
}

/* ---------------------------------------------------------------------- */
/* Counter-based random decisions: SplitMix64 (Steele, Lea, Flood, OOPSLA  */
/* 2014).  Draw k of a stream seeded with `seed` is the output of the      */
/* generator after k+1 increments of its state by the golden gamma.        */
/* ---------------------------------------------------------------------- */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double oracle_uniform(uint64_t seed, uint64_t k)
{
    return (double)(oracle_splitmix64(seed, k) >> 11) * 0x1.0p-53;
}

/* ---------------------------------------------------------------------- */
/* Tile norms (Sec. 3: the criteria use the 1-norm of each tile).          */
/* ---------------------------------------------------------------------- */
double oracle_tile_norm1(const double *A, int64_t lda, int64_t rows, int64_t cols)
{
    double best = 0.0;
    for (int64_t j = 0; j < cols; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < rows; ++i) s += fabs(A[IX(i, j, lda)]);
        if (isnan(s)) return s;
        if (s > best) best = s;
    }
    return best;
}

static double tile_maxabs(const double *A, int64_t lda, int64_t rows, int64_t cols)
{
    double best = 0.0;
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t i = 0; i < rows; ++i) {
            double a = fabs(A[IX(i, j, lda)]);
            if (a > best) best = a;
        }
    return best;
}

/* ---------------------------------------------------------------------- */
/* GETRF: textbook right-looking Gaussian elimination with partial         */
/* pivoting on one m x m tile (Alg. 2, Factor).  The pivot is the first    */
/* row holding the largest magnitude of the remaining column.  A column    */
/* that is exactly zero is skipped (no interchange, no scaling) and         */
/* reported.  Returns the 1-based index of the first zero pivot, 0 if none. */
/* ---------------------------------------------------------------------- */
/* The same elimination on a tall rows x cols block (rows >= cols): the     */
/* pivot of column c is searched over rows c..rows-1 (the diagonal domain   */
/* of Sec. 2.1 stacks several tiles of the panel).                          */
static int64_t gepp_rect(int64_t rows, int64_t cols, double *W, int64_t ldw, int32_t *ipiv)
{
    int64_t first_zero = 0;
    for (int64_t c = 0; c < cols; ++c) {
        int64_t p = c;
        double best = fabs(W[IX(c, c, ldw)]);
        for (int64_t r = c + 1; r < rows; ++r) {
            double a = fabs(W[IX(r, c, ldw)]);
            if (a > best) { best = a; p = r; }
        }
        ipiv[c] = (int32_t)p;
        if (best == 0.0) {
            if (!first_zero) first_zero = c + 1;
            continue;
        }
        if (p != c)
            for (int64_t j = 0; j < cols; ++j) {
                double t = W[IX(c, j, ldw)];
                W[IX(c, j, ldw)] = W[IX(p, j, ldw)];
                W[IX(p, j, ldw)] = t;
            }
        double piv = W[IX(c, c, ldw)];
        for (int64_t r = c + 1; r < rows; ++r) W[IX(r, c, ldw)] /= piv;
        for (int64_t j = c + 1; j < cols; ++j) {
            double u = W[IX(c, j, ldw)];
            for (int64_t r = c + 1; r < rows; ++r) W[IX(r, j, ldw)] -= W[IX(r, c, ldw)] * u;
        }
    }
    return first_zero;
}

int64_t oracle_gepp(int64_t m, double *W, int64_t ldw, int32_t *ipiv)
{
    return gepp_rect(m, m, W, ldw, ipiv);
}

/* ---------------------------------------------------------------------- */
/* Diagonal domain of step k (Sec. 2.1, last paragraph; Sec. 3.1 and 3.3):  */
/* the panel tiles held by the node that holds A_kk when tile rows are      */
/* dealt cyclically over p rows of nodes, i.e. the tiles i >= k with        */
/* i = k (mod p), in increasing order (tiles[0] = k).  p = 0: the diagonal  */
/* tile alone.  The domain's tiles are stacked in that order; stacked row s */
/* is row s % nb of tile tiles[s / nb] (only the last tile of the matrix   */
/* can be short, and it comes last).                                        */
/* ---------------------------------------------------------------------- */
static int64_t domain_tiles(int64_t k, int64_t n, int64_t p, int64_t *tiles)
{
    int64_t d = 0;
    tiles[d++] = k;
    if (p > 0)
        for (int64_t i = k + p; i < n; i += p) tiles[d++] = i;
    return d;
}

static int64_t domain_row(int64_t s, const int64_t *tiles, int64_t nb)
{
    return tiles[s / nb] * nb + s % nb;
}

/* Row interchanges of a domain factorization, in order, on columns c0..c1-1
 * of the N x * matrix X: stacked row c <-> stacked row dpiv[c]. */
static void domain_swap(int64_t mk, const int32_t *dpiv, const int64_t *tiles, int64_t nb,
                        double *X, int64_t ldx, int64_t c0, int64_t c1)
{
    for (int64_t c = 0; c < mk; ++c) {
        if (dpiv[c] == c) continue;
        int64_t a = domain_row(c, tiles, nb), b = domain_row(dpiv[c], tiles, nb);
        for (int64_t j = c0; j < c1; ++j) {
            double t = X[IX(a, j, ldx)]; X[IX(a, j, ldx)] = X[IX(b, j, ldx)]; X[IX(b, j, ldx)] = t;
        }
    }
}

/* ||W^{-1}||_1 from the factors P W = L U: column j of W^{-1} solves
 * L U x = P e_j (Sec. 3.4 notes the inverse norm is obtained from L and U;
 * here it is computed exactly, column by column). */
double oracle_inv_norm1(int64_t m, const double *LU, int64_t ldw, const int32_t *ipiv)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    double best = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t r = 0; r < m; ++r) x[r] = (r == j) ? 1.0 : 0.0;
        for (int64_t c = 0; c < m; ++c) { /* x <- P x, interchanges in order */
            int64_t p = ipiv[c];
            double t = x[c]; x[c] = x[p]; x[p] = t;
        }
        for (int64_t c = 0; c < m; ++c) /* L y = x (unit lower) */
            for (int64_t r = c + 1; r < m; ++r) x[r] -= LU[IX(r, c, ldw)] * x[c];
        for (int64_t c = m - 1; c >= 0; --c) { /* U z = y */
            x[c] /= LU[IX(c, c, ldw)];
            for (int64_t r = 0; r < c; ++r) x[r] -= LU[IX(r, c, ldw)] * x[c];
        }
        double s = 0.0;
        for (int64_t r = 0; r < m; ++r) s += fabs(x[r]);
        if (s > best || isnan(s)) best = s;
    }
    free(x);
    return best;
}

/* Products with B = U^{-1} L^{-1} (the inverse of P W up to the column
 * permutation, which leaves the 1-norm unchanged) and with B^T, from the
 * factors L\U in place: triangular solves in the plain loop order.        */
static void est_apply(int64_t m, const double *LU, int64_t ldw, double *x, int transpose)
{
    if (!transpose) {
        for (int64_t c = 0; c < m; ++c) /* L t = x (unit lower) */
            for (int64_t r = c + 1; r < m; ++r) x[r] -= LU[IX(r, c, ldw)] * x[c];
        for (int64_t c = m - 1; c >= 0; --c) { /* U y = t */
            x[c] /= LU[IX(c, c, ldw)];
            for (int64_t r = 0; r < c; ++r) x[r] -= LU[IX(r, c, ldw)] * x[c];
        }
    } else {
        for (int64_t r = 0; r < m; ++r) { /* U^T t = x */
            double v = x[r];
            for (int64_t c = 0; c < r; ++c) v -= LU[IX(c, r, ldw)] * x[c];
            x[r] = v / LU[IX(r, r, ldw)];
        }
        for (int64_t r = m - 1; r >= 0; --r) { /* L^T z = t (unit lower) */
            double v = x[r];
            for (int64_t c = r + 1; c < m; ++c) v -= LU[IX(c, r, ldw)] * x[c];
            x[r] = v;
        }
    }
}

static double est_norm1(int64_t m, const double *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += fabs(x[i]);
    return s;
}

static int64_t est_argmax(int64_t m, const double *x) /* first index of the largest |x_i| */
{
    int64_t j = 0;
    for (int64_t i = 1; i < m; ++i)
        if (fabs(x[i]) > fabs(x[j])) j = i;
    return j;
}

/* Estimate of ||W^{-1}||_1 in O(m^2) per iteration from the factors P W = L U
 * (Sec. 3.4: the inverse norm costs a few triangular solves when estimated):
 * Hager's method with Higham's refinements, the iteration LAPACK runs for its
 * condition estimates.  With B = W^{-1}:
 *   x = (1/m, ..., 1/m); y = B x; est = ||y||_1; xi = sign(y); z = B^T xi;
 *   up to four times: j = the first index of max |z|, y = B e_j,
 *   est = ||y||_1; stop if sign(y) repeats xi or est did not grow (the new
 *   value stands, as in Higham's algorithm); else xi = sign(y), z = B^T xi,
 *   and stop when the previous j already attains it (z_jlast == ||z||_inf);
 *   finally x_i = (-1)^i (1 + i/(m-1)), est = max(est, 2 ||B x||_1 / (3m)).
 * sign(0) = +1.  The result is a lower bound of ||W^{-1}||_1 (every est is
 * ||B x||_1 for some ||x||_1 <= 1).                                        */
double oracle_inv_norm1_est(int64_t m, const double *LU, int64_t ldw)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    int *xi = (int *)malloc((size_t)m * sizeof(int));
    for (int64_t i = 0; i < m; ++i) x[i] = 1.0 / (double)m;
    est_apply(m, LU, ldw, x, 0);
    double est = est_norm1(m, x);
    if (m > 1) {
        for (int64_t i = 0; i < m; ++i) { xi[i] = x[i] >= 0.0 ? 1 : -1; x[i] = (double)xi[i]; }
        est_apply(m, LU, ldw, x, 1);
        int64_t j = est_argmax(m, x);
        int iter = 2;
        for (;;) {
            for (int64_t i = 0; i < m; ++i) x[i] = (i == j) ? 1.0 : 0.0;
            est_apply(m, LU, ldw, x, 0);
            const double estold = est;
            est = est_norm1(m, x);
            int same = 1;
            for (int64_t i = 0; i < m; ++i) same &= ((x[i] >= 0.0 ? 1 : -1) == xi[i]);
            if (same) break;               /* repeated sign vector: converged */
            if (est <= estold) break;      /* no growth: cycling (the new value stands) */
            for (int64_t i = 0; i < m; ++i) { xi[i] = x[i] >= 0.0 ? 1 : -1; x[i] = (double)xi[i]; }
            est_apply(m, LU, ldw, x, 1);
            const int64_t jlast = j;
            j = est_argmax(m, x);
            if (x[jlast] == fabs(x[j]) || iter >= 5) break;
            ++iter;
        }
        for (int64_t i = 0; i < m; ++i) x[i] = (i % 2 ? -1.0 : 1.0) * (1.0 + (double)i / (double)(m - 1));
        est_apply(m, LU, ldw, x, 0);
        const double alt = 2.0 * est_norm1(m, x) / (3.0 * (double)m);
        if (alt > est) est = alt;
    }
    free(x); free(xi);
    return est;
}

/* ||A^{-1}||_1 of an m x m tile from its GEQRT factors (variant A2, Sec.
 * 2.3: A = Q U with Q given by the unit-lower reflectors V and the compact-WY
 * factor T, U upper triangular).  By definition A^{-1} = U^{-1} Q^T: Q^T is
 * formed by applying the reflectors to the identity, then every column is
 * back-substituted with U, and the largest absolute column sum is returned.
 * VR holds V below the diagonal and U on and above it; U must have no zero
 * on its diagonal. */
void oracle_unmqr(int64_t mk, const double *V, int64_t ldv, const double *T, int64_t ldt,
                  int64_t nc, double *C, int64_t ldc);
double oracle_inv_norm1_qr(int64_t m, const double *VR, int64_t ldv, const double *T, int64_t ldt)
{
    double *X = (double *)calloc((size_t)(m > 0 ? m * m : 1), sizeof(double));
    for (int64_t i = 0; i < m; ++i) X[IX(i, i, m)] = 1.0;
    oracle_unmqr(m, VR, ldv, T, ldt, m, X, m);
    double best = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t c = m - 1; c >= 0; --c) {
            const double x = X[IX(c, j, m)] / VR[IX(c, c, ldv)];
            X[IX(c, j, m)] = x;
            for (int64_t r = 0; r < c; ++r) X[IX(r, j, m)] -= VR[IX(r, c, ldv)] * x;
        }
        double sum = 0.0;
        for (int64_t i = 0; i < m; ++i) sum += fabs(X[IX(i, j, m)]);
        if (sum > best || isnan(sum)) best = sum;
    }
    free(X);
    return best;
}

/* ---------------------------------------------------------------------- */
/* Householder reflector (Golub & Van Loan, Sec. 5.1, with the LAPACK sign  */
/* convention): given alpha and the tail x of length len, find beta, tau,  */
/* v = [1; x/(alpha-beta)] with (I - tau v v^T) [alpha; x] = [beta; 0].     */
/* beta = -sign(alpha) ||[alpha;x]||_2, sign(0) = +1; tau = 0 (H = I) when  */
/* the tail is exactly zero.  On exit *alpha = beta and x holds the tail   */
/* of v.  xs is the stride of x.                                           */
/* ---------------------------------------------------------------------- */
static double householder(double *alpha, double *x, int64_t len, int64_t xs)
{
    double ss = 0.0;
    for (int64_t r = 0; r < len; ++r) ss += x[r * xs] * x[r * xs];
    if (ss == 0.0) return 0.0;
    double a = *alpha;
    double norm = sqrt(a * a + ss);
    double beta = (a >= 0.0) ? -norm : norm;
    double tau = (beta - a) / beta;
    double scal = 1.0 / (a - beta);
    for (int64_t r = 0; r < len; ++r) x[r * xs] *= scal;
    *alpha = beta;
    return tau;
}

/* GEQRT on an m x m tile: A = Q R with Q = H_0 H_1 ... H_{m-1} = I - V T V^T,
 * V unit lower triangular stored below the diagonal, R on and above it,
 * T upper triangular (Schreiber & Van Loan compact WY). */
void oracle_geqrt(int64_t m, double *A, int64_t lda, double *T, int64_t ldt)
{
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i) T[IX(i, j, ldt)] = 0.0;
    double *w = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    for (int64_t c = 0; c < m; ++c) {
        double tau = householder(&A[IX(c, c, lda)], &A[IX(c + 1, c, lda)], m - c - 1, 1);
        /* apply H_c = I - tau v v^T to columns c+1..m-1 */
        for (int64_t j = c + 1; j < m; ++j) {
            double s = A[IX(c, j, lda)];
            for (int64_t r = c + 1; r < m; ++r) s += A[IX(r, c, lda)] * A[IX(r, j, lda)];
            s *= tau;
            A[IX(c, j, lda)] -= s;
            for (int64_t r = c + 1; r < m; ++r) A[IX(r, j, lda)] -= A[IX(r, c, lda)] * s;
        }
        /* T(0:c, c) = -tau T(0:c,0:c) V(:,0:c)^T v_c ; T(c,c) = tau */
        for (int64_t l = 0; l < c; ++l) { /* w_l = v_l^T v_c, v_l has 1 at row l */
            double s = A[IX(c, l, lda)]; /* v_l(c) * v_c(c)=1 */
            for (int64_t r = c + 1; r < m; ++r) s += A[IX(r, l, lda)] * A[IX(r, c, lda)];
            w[l] = s;
        }
        for (int64_t l = 0; l < c; ++l) {
            double s = 0.0;
            for (int64_t q = l; q < c; ++q) s += T[IX(l, q, ldt)] * w[q];
            T[IX(l, c, ldt)] = -tau * s;
        }
        T[IX(c, c, ldt)] = tau;
    }
    free(w);
}

/* UNMQR: C <- Q^T C = C - V T^T (V^T C) for the reflectors of a GEQRT tile
 * (m_k x m_k V, unit lower) applied to an m_k x nc tile C. */
void oracle_unmqr(int64_t mk, const double *V, int64_t ldv, const double *T, int64_t ldt,
                  int64_t nc, double *C, int64_t ldc)
{
    double *W = (double *)malloc((size_t)(mk > 0 ? mk : 1) * sizeof(double));
    for (int64_t j = 0; j < nc; ++j) {
        for (int64_t l = 0; l < mk; ++l) { /* W = V^T C(:,j) */
            double s = C[IX(l, j, ldc)];
            for (int64_t r = l + 1; r < mk; ++r) s += V[IX(r, l, ldv)] * C[IX(r, j, ldc)];
            W[l] = s;
        }
        for (int64_t l = mk - 1; l >= 0; --l) { /* W = T^T W (T upper => T^T lower) */
            double s = 0.0;
            for (int64_t q = 0; q <= l; ++q) s += T[IX(q, l, ldt)] * W[q];
            W[l] = s;
        }
        for (int64_t l = 0; l < mk; ++l) { /* C -= V W */
            C[IX(l, j, ldc)] -= W[l];
            for (int64_t r = l + 1; r < mk; ++r) C[IX(r, j, ldc)] -= V[IX(r, l, ldv)] * W[l];
        }
    }
    free(W);
}

/* TSQRT: QR of [R; A] with R (m_k x m_k) upper triangular and A (m_i x m_k)
 * dense.  Reflector c is v_c = [e_c ; y_c]; the tails y_c overwrite A,
 * R is updated in place and T is the compact-WY factor of the m_k
 * reflectors (the e_c parts are orthogonal, so only Y enters T). */
void oracle_tsqrt(int64_t mk, double *R, int64_t ldr, int64_t mi, double *A, int64_t lda,
                  double *T, int64_t ldt)
{
    for (int64_t j = 0; j < mk; ++j)
        for (int64_t i = 0; i < mk; ++i) T[IX(i, j, ldt)] = 0.0;
    double *w = (double *)malloc((size_t)(mk > 0 ? mk : 1) * sizeof(double));
    for (int64_t c = 0; c < mk; ++c) {
        double tau = householder(&R[IX(c, c, ldr)], &A[IX(0, c, lda)], mi, 1);
        for (int64_t j = c + 1; j < mk; ++j) {
            double s = R[IX(c, j, ldr)];
            for (int64_t r = 0; r < mi; ++r) s += A[IX(r, c, lda)] * A[IX(r, j, lda)];
            s *= tau;
            R[IX(c, j, ldr)] -= s;
            for (int64_t r = 0; r < mi; ++r) A[IX(r, j, lda)] -= A[IX(r, c, lda)] * s;
        }
        for (int64_t l = 0; l < c; ++l) {
            double s = 0.0;
            for (int64_t r = 0; r < mi; ++r) s += A[IX(r, l, lda)] * A[IX(r, c, lda)];
            w[l] = s;
        }
        for (int64_t l = 0; l < c; ++l) {
            double s = 0.0;
            for (int64_t q = l; q < c; ++q) s += T[IX(l, q, ldt)] * w[q];
            T[IX(l, c, ldt)] = -tau * s;
        }
        T[IX(c, c, ldt)] = tau;
    }
    free(w);
}

/* TSMQR: [Ck; Ci] <- Q^T [Ck; Ci] for the TSQRT reflectors V = [I; Y]:
 * W = T^T (Ck + Y^T Ci); Ck -= W; Ci -= Y W. */
void oracle_tsmqr(int64_t mk, int64_t mi, const double *Y, int64_t ldy, const double *T, int64_t ldt,
                  int64_t nc, double *Ck, int64_t ldck, double *Ci, int64_t ldci)
{
    double *W = (double *)malloc((size_t)(mk > 0 ? mk : 1) * sizeof(double));
    for (int64_t j = 0; j < nc; ++j) {
        for (int64_t l = 0; l < mk; ++l) {
            double s = Ck[IX(l, j, ldck)];
            for (int64_t r = 0; r < mi; ++r) s += Y[IX(r, l, ldy)] * Ci[IX(r, j, ldci)];
            W[l] = s;
        }
        for (int64_t l = mk - 1; l >= 0; --l) {
            double s = 0.0;
            for (int64_t q = 0; q <= l; ++q) s += T[IX(q, l, ldt)] * W[q];
            W[l] = s;
        }
        for (int64_t l = 0; l < mk; ++l) Ck[IX(l, j, ldck)] -= W[l];
        for (int64_t l = 0; l < mk; ++l)
            for (int64_t r = 0; r < mi; ++r) Ci[IX(r, j, ldci)] -= Y[IX(r, l, ldy)] * W[l];
    }
    free(W);
}

/* TTQRT (Alg. 4b): QR of [R1; R2] with both m_k x m_k upper triangular.
 * Reflector c is v_c = [e_c; y_c] with y_c = R2(0..c, c) (zero below row c,
 * so the tails stay upper triangular and overwrite R2's upper triangle); R1
 * is updated in place and T is the compact-WY factor of the m_k
 * reflectors.  Equal to TSQRT on a triangular R2 with the zero products
 * left out. */
void oracle_ttqrt(int64_t mk, double *R1, int64_t ld1, double *R2, int64_t ld2, double *T, int64_t ldt)
{
    for (int64_t j = 0; j < mk; ++j)
        for (int64_t i = 0; i < mk; ++i) T[IX(i, j, ldt)] = 0.0;
    double *w = (double *)malloc((size_t)(mk > 0 ? mk : 1) * sizeof(double));
    for (int64_t c = 0; c < mk; ++c) {
        double tau = householder(&R1[IX(c, c, ld1)], &R2[IX(0, c, ld2)], c + 1, 1);
        for (int64_t j = c + 1; j < mk; ++j) {
            double s = R1[IX(c, j, ld1)];
            for (int64_t r = 0; r <= c; ++r) s += R2[IX(r, c, ld2)] * R2[IX(r, j, ld2)];
            s *= tau;
            R1[IX(c, j, ld1)] -= s;
            for (int64_t r = 0; r <= c; ++r) R2[IX(r, j, ld2)] -= R2[IX(r, c, ld2)] * s;
        }
        for (int64_t l = 0; l < c; ++l) { /* w_l = y_l^T y_c, y_l zero below row l */
            double s = 0.0;
            for (int64_t r = 0; r <= l; ++r) s += R2[IX(r, l, ld2)] * R2[IX(r, c, ld2)];
            w[l] = s;
        }
        for (int64_t l = 0; l < c; ++l) {
            double s = 0.0;
            for (int64_t q = l; q < c; ++q) s += T[IX(l, q, ldt)] * w[q];
            T[IX(l, c, ldt)] = -tau * s;
        }
        T[IX(c, c, ldt)] = tau;
    }
    free(w);
}

/* TTMQR: [C1; C2] <- Q^T [C1; C2] for the TTQRT reflectors V = [I; Y], Y
 * upper triangular (its upper triangle in Y, entries below ignored):
 * W = T^T (C1 + Y^T C2); C1 -= W; C2 -= Y W. */
void oracle_ttmqr(int64_t mk, const double *Y, int64_t ldy, const double *T, int64_t ldt,
                  int64_t nc, double *C1, int64_t ld1, double *C2, int64_t ld2)
{
    double *W = (double *)malloc((size_t)(mk > 0 ? mk : 1) * sizeof(double));
    for (int64_t j = 0; j < nc; ++j) {
        for (int64_t l = 0; l < mk; ++l) {
            double s = C1[IX(l, j, ld1)];
            for (int64_t r = 0; r <= l; ++r) s += Y[IX(r, l, ldy)] * C2[IX(r, j, ld2)];
            W[l] = s;
        }
        for (int64_t l = mk - 1; l >= 0; --l) {
            double s = 0.0;
            for (int64_t q = 0; q <= l; ++q) s += T[IX(q, l, ldt)] * W[q];
            W[l] = s;
        }
        for (int64_t l = 0; l < mk; ++l) C1[IX(l, j, ld1)] -= W[l];
        for (int64_t l = 0; l < mk; ++l)
            for (int64_t r = 0; r <= l; ++r) C2[IX(r, j, ld2)] -= Y[IX(r, l, ldy)] * W[l];
    }
    free(W);
}

/* The elimination tree of a QR step (Sec. 2.2, Alg. 3; the two-level
 * reduction of Sec. 2.2 and 4.2): the panel tiles k..n-1 form groups of S
 * consecutive tiles (S = qr_tree; S <= 0 or S >= n-k: one group, the flat
 * tree), a trailing group of a single tile joining the group before it.
 * Within a group its first tile (the head) eliminates the others with TS
 * kernels (Alg. 4a); then the heads are reduced by a binary tree of TT
 * kernels (Alg. 4b): at distance d = 1, 2, 4, .., head g eliminates head
 * g + d for g = 0, 2d, 4d, ...  head[0..G-1] receive the heads, head[G] = n;
 * returns G. */
static int64_t qr_groups(int64_t k, int64_t n, int32_t S, int64_t *head)
{
    const int64_t m = n - k;
    const int64_t s = (S <= 0 || S >= m) ? m : S;
    int64_t G = (m + s - 1) / s;
    if (G > 1 && m - (G - 1) * s == 1) --G;
    for (int64_t g = 0; g < G; ++g) head[g] = k + g * s;
    head[G] = n;
    return G;
}

/* LU-step kernels of Alg. 2. */
/* Eliminate: X <- X U^{-1} (U upper, non-unit), X is mi x mk. */
static void trsm_right_upper(int64_t mk, const double *U, int64_t ldu, int64_t mi, double *X, int64_t ldx)
{
    for (int64_t c = 0; c < mk; ++c) {
        for (int64_t l = 0; l < c; ++l) {
            double u = U[IX(l, c, ldu)];
            for (int64_t r = 0; r < mi; ++r) X[IX(r, c, ldx)] -= X[IX(r, l, ldx)] * u;
        }
        double d = U[IX(c, c, ldu)];
        for (int64_t r = 0; r < mi; ++r) X[IX(r, c, ldx)] /= d;
    }
}

/* Apply: X <- L^{-1} P X, L unit lower (stored below the diagonal of LU). */
static void swptrsm(int64_t mk, const double *LU, int64_t ldw, const int32_t *ipiv,
                    int64_t nc, double *X, int64_t ldx)
{
    for (int64_t j = 0; j < nc; ++j) {
        for (int64_t c = 0; c < mk; ++c) {
            int64_t p = ipiv[c];
            double t = X[IX(c, j, ldx)]; X[IX(c, j, ldx)] = X[IX(p, j, ldx)]; X[IX(p, j, ldx)] = t;
        }
        for (int64_t c = 0; c < mk; ++c)
            for (int64_t r = c + 1; r < mk; ++r) X[IX(r, j, ldx)] -= LU[IX(r, c, ldw)] * X[IX(c, j, ldx)];
    }
}

/* Update: C <- C - A B, C mi x nc, A mi x mk, B mk x nc. */
static void gemm_minus(int64_t mi, int64_t nc, int64_t mk, const double *A, int64_t lda,
                       const double *B, int64_t ldb, double *C, int64_t ldc)
{
    for (int64_t j = 0; j < nc; ++j)
        for (int64_t l = 0; l < mk; ++l) {
            double b = B[IX(l, j, ldb)];
            for (int64_t r = 0; r < mi; ++r) C[IX(r, j, ldc)] -= A[IX(r, l, lda)] * b;
        }
}

/* Table 1 work of step k with r = n-k-1 trailing tiles, in units of nb^3.
 * Variant A2 (Sec. 2.3) doubles the Factor (GEQRT instead of GETRF) and the
 * Apply (ORMQR instead of TRSM) of an LU step: 4/3 + 3r + 2r^2. */
static double step_units_v(int64_t r, int is_qr, int a2)
{
    double u = 2.0 / 3.0 + 2.0 * (double)r + 2.0 * (double)r * (double)r;
    if (is_qr) return 2.0 * u;
    return a2 ? u + 2.0 / 3.0 + (double)r : u;
}
static double step_units(int64_t r, int is_qr) { return step_units_v(r, is_qr, 0); }

/* ---------------------------------------------------------------------- */
/* The hybrid LU-QR factorization (Alg. 1).                                */
/*   criterion/alpha  robustness test (Sec. 3); forced: n decisions for    */
/*                    CRIT_FORCED; seed for CRIT_RANDOM.                   */
/*   mumps_reading    0: est(j) = away(j) prod_{i<j} gf(i) (primary);       */
/*                    1: est(j) = away(j) gf(j); 2: est(j) = away(j) prod_i gf(i) */
/*   nsteps           number of panel steps to run (<0: all).              */
/*   B (N x nrhs)     if non-NULL, transformed along with A (augmented      */
/*                    system of Sec. 2.4); after the last step it holds     */
/*                    the forward-transformed right-hand sides.            */
/* Outputs ipiv, Tq, dec, s, m, margin may each be NULL.                   */
/* ---------------------------------------------------------------------- */
/*   domain_stride    p of the diagonal domain (see domain_tiles); 0: the  */
/*                    diagonal tile alone.  With a domain of more than one  */
/*                    tile the LU attempt is GEPP on the stacked domain,    */
/*                    the criterion sees A_kk and the sub-diagonal tiles    */
/*                    after its interchanges (Sec. 3.1), an LU step applies */
/*                    them to the trailing columns of the domain's rows and */
/*                    stores the domain's multipliers, and ipiv[k*nb + c]   */
/*                    holds the stacked row exchanged at column c.          */
/*   lu_variant       0 or 1: LU steps of variant A1 (Alg. 2, GEPP on a     */
/*                    backup copy); 2: variant A2 (Sec. 2.3): every step    */
/*                    starts with GEQRT of A_kk in place, the criterion     */
/*                    takes ||A_kk^{-1}||_1 from those factors, an LU step  */
/*                    eliminates with U = R and applies Q^T, and a QR step  */
/*                    continues from the same GEQRT.  A2 is defined for the */
/*                    Max, Sum, Random and Forced criteria without a domain */
/*                    or the estimate (-23 otherwise).                      */
/*   qr_tree          0: every QR step is the flat TS tree (Alg. 4a, the     */
/*                    eliminator of every A_ik is A_kk); S > 0: groups of S   */
/*                    tiles reduced by TS, their heads by a binary TT tree    */
/*                    (qr_groups); Tt (n*n blocks of nb*nb, required then)    */
/*                    receives the TT factors.                               */
int oracle_factor_t(int64_t N, double *A, int64_t lda, int64_t nb, int32_t criterion, double alpha,
                    uint64_t seed, const int8_t *forced, int32_t mumps_reading, int64_t nsteps,
                    double *B, int64_t ldb, int64_t nrhs,
                    int32_t *ipiv, double *Tq, int8_t *dec, double *s_out, double *m_out,
                    double *margin_out, double *diag, int32_t domain_stride, int32_t invnorm_estimate,
                    int32_t lu_variant, int32_t qr_tree, double *Tt)
{
    if (N < 1) return -1;
    if (nb < 1) return -4;
    if (lda < N) return -3;
    if (!(alpha >= 0.0)) return -6;
    if (criterion < 0 || criterion > 4) return -5;
    if (criterion == CRIT_FORCED && !forced) return -8;
    if (B && ldb < N) return -12;
    if (domain_stride < 0) return -21;
    if (lu_variant < 0 || lu_variant > 2) return -22;
    const int a2 = lu_variant == 2;
    if (a2 && (domain_stride > 0 || invnorm_estimate || criterion == CRIT_MUMPS)) return -23;
    if (qr_tree < 0) return -24;
    if (qr_tree > 0 && !Tt) return -25;

    const int64_t n = (N + nb - 1) / nb;
    if (nsteps < 0 || nsteps > n) nsteps = n;

    int32_t *piv = (int32_t *)calloc((size_t)nb, sizeof(int32_t));
    double *W = (double *)malloc((size_t)nb * (size_t)nb * sizeof(double));
    double *Tloc = (double *)malloc((size_t)nb * (size_t)nb * sizeof(double));
    double *colsum_scratch = (double *)malloc((size_t)nb * sizeof(double));
    double *away = (double *)malloc((size_t)nb * sizeof(double));
    double *lmax = (double *)malloc((size_t)nb * sizeof(double));
    double *nrm_before = diag ? (double *)malloc((size_t)n * (size_t)n * sizeof(double)) : NULL;
    (void)colsum_scratch;
    int64_t *dtile = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    double *Wd = domain_stride > 0 ? (double *)malloc((size_t)N * (size_t)nb * sizeof(double)) : NULL;
    double *Pd = domain_stride > 0 ? (double *)malloc((size_t)N * (size_t)nb * sizeof(double)) : NULL;
    int32_t *dpiv = (int32_t *)calloc((size_t)nb, sizeof(int32_t));
    int64_t *ghead = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));

    if (diag) {
        for (int q = 0; q < DG_COUNT; ++q) diag[q] = 0.0;
    }
    double max_tile0 = 0.0, max_elem0 = 0.0, max_tile = 0.0, max_elem = 0.0;

    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t mk = tsize(N, nb, k);
        double *Akk = &A[IX(k * nb, k * nb, lda)];

        /* diagnostics: growth over the active submatrix at the start of step k */
        if (diag) {
            for (int64_t j = k; j < n; ++j)
                for (int64_t i = k; i < n; ++i) {
                    const double *Aij = &A[IX(i * nb, j * nb, lda)];
                    double t = oracle_tile_norm1(Aij, lda, tsize(N, nb, i), tsize(N, nb, j));
                    double e = tile_maxabs(Aij, lda, tsize(N, nb, i), tsize(N, nb, j));
                    nrm_before[IX(i, j, n)] = t;
                    if (t > max_tile) max_tile = t;
                    if (e > max_elem) max_elem = e;
                }
            if (k == 0) { max_tile0 = max_tile; max_elem0 = max_elem; }
        }

        const int64_t d = domain_tiles(k, n, domain_stride, dtile);
        const int64_t R = (d - 1) * nb + tsize(N, nb, dtile[d - 1]);  /* rows of the stacked domain */
        double *Tkk = Tq ? &Tq[((size_t)k * n + k) * nb * nb] : Tloc;
        int64_t zero_piv;
        if (a2) {
            /* ---- Factor, variant A2 (Sec. 2.3): A_kk = Q_kk U_kk by GEQRT in
             * place (V below the diagonal, U on and above it); no backup.  A
             * zero on the diagonal of U marks a singular tile, as a zero GEPP
             * pivot does in A1. */
            oracle_geqrt(mk, Akk, lda, Tkk, nb);
            zero_piv = 0;
            for (int64_t c = 0; c < mk && !zero_piv; ++c)
                if (Akk[IX(c, c, lda)] == 0.0) zero_piv = c + 1;
        } else if (d == 1) {
        /* ---- Factor: backup copy W of A_kk, GEPP on the copy (Sec. 4, Backup Panel / LU On Panel) */
        for (int64_t j = 0; j < mk; ++j)
            for (int64_t i = 0; i < mk; ++i) W[IX(i, j, nb)] = Akk[IX(i, j, lda)];
        for (int64_t j = 0; j < mk; ++j) { /* MUMPS: local column maxima before factoring */
            double b = 0.0;
            for (int64_t i = 0; i < mk; ++i) { double a = fabs(Akk[IX(i, j, lda)]); if (a > b) b = a; }
            lmax[j] = b;
        }
        zero_piv = oracle_gepp(mk, W, nb, piv);
        } else {
            /* ---- Factor on the diagonal domain: GEPP on a copy of the stacked
             * domain tiles; W receives its top block L11\U (the diagonal tile
             * after the domain's interchanges, Sec. 3.1), whose own pivots are
             * then the identity. */
            for (int64_t j = 0; j < mk; ++j)
                for (int64_t r = 0; r < R; ++r) Wd[IX(r, j, R)] = A[IX(domain_row(r, dtile, nb), k * nb + j, lda)];
            memcpy(Pd, Wd, (size_t)R * (size_t)mk * sizeof(double));
            for (int64_t j = 0; j < mk; ++j) { /* MUMPS: local column maxima over the domain */
                double b = 0.0;
                for (int64_t r = 0; r < R; ++r) { double a = fabs(Wd[IX(r, j, R)]); if (a > b) b = a; }
                lmax[j] = b;
            }
            zero_piv = gepp_rect(R, mk, Wd, R, dpiv);
            for (int64_t j = 0; j < mk; ++j)
                for (int64_t i = 0; i < mk; ++i) W[IX(i, j, nb)] = Wd[IX(i, j, R)];
            for (int64_t c = 0; c < mk; ++c) piv[c] = (int32_t)c;
            /* the original panel values of the domain, permuted like the rows of Wd */
            for (int64_t c = 0; c < mk; ++c)
                if (dpiv[c] != c)
                    for (int64_t j = 0; j < mk; ++j) {
                        double t = Pd[IX(c, j, R)]; Pd[IX(c, j, R)] = Pd[IX(dpiv[c], j, R)]; Pd[IX(dpiv[c], j, R)] = t;
                    }
        }

        /* ---- Check: criterion inputs (Sec. 3) */
        double s = 0.0, m = 0.0;
        int nonfinite = 0;
        if (!zero_piv) {
            /* ||A_kk^{-1}||_1 exactly, or its O(n_b^2) estimate (Sec. 3.4) */
            double inv = a2 ? oracle_inv_norm1_qr(mk, Akk, lda, Tkk, nb)
                       : invnorm_estimate ? oracle_inv_norm1_est(mk, W, nb) : oracle_inv_norm1(mk, W, nb, piv);
            s = 1.0 / inv;
        }
        for (int64_t j = 0; j < mk; ++j) away[j] = 0.0;
        for (int64_t i = k + 1, t_dom = 1; i < n; ++i) {
            const double *Aik = &A[IX(i * nb, k * nb, lda)];
            int64_t mi = tsize(N, nb, i);
            const int in_domain = t_dom < d && dtile[t_dom] == i;
            double t = in_domain ? oracle_tile_norm1(&Pd[IX(t_dom * nb, 0, R)], R, mi, mk)
                                 : oracle_tile_norm1(Aik, lda, mi, mk);
            if (criterion == CRIT_SUM) m += t;
            else if (t > m || isnan(t)) m = t;
            if (in_domain) { ++t_dom; continue; } /* MUMPS: away_max is over the tiles off the domain */
            for (int64_t j = 0; j < mk; ++j)
                for (int64_t r = 0; r < mi; ++r) {
                    double a = fabs(Aik[IX(r, j, lda)]);
                    if (a > away[j] || isnan(a)) away[j] = a;
                }
        }
        if (!isfinite(s) || !isfinite(m)) nonfinite = 1;

        /* ---- Decision */
        int lu;
        double margin;
        if (criterion == CRIT_FORCED) {
            lu = forced[k] != 0;
            margin = lu ? 1.0 : -1.0;
        } else if (isinf(alpha)) {
            lu = 1; margin = 1.0;
        } else if (alpha == 0.0) {
            lu = 0; margin = -1.0;
        } else if (zero_piv) {
            lu = 0; margin = -1.0;
        } else if (criterion == CRIT_MAX || criterion == CRIT_SUM) {
            if (nonfinite) { lu = 0; margin = -1.0; }
            else {
                double as = alpha * s;
                lu = (as >= m);
                double den = as > m ? as : m;
                if (den < DBL_MIN) den = DBL_MIN;
                margin = (as - m) / den;
            }
        } else if (criterion == CRIT_MUMPS) {
            lu = 1; margin = INFINITY;
            double prod_all = 1.0;
            for (int64_t j = 0; j < mk; ++j) prod_all *= fabs(W[IX(j, j, nb)]) / lmax[j];
            double prod = 1.0;
            double smin = INFINITY, emax = 0.0;
            for (int64_t j = 0; j < mk; ++j) {
                double pivj = fabs(W[IX(j, j, nb)]);
                double gfj = pivj / lmax[j];
                double est;
                if (mumps_reading == 1) est = away[j] * gfj;
                else if (mumps_reading == 2) est = away[j] * prod_all;
                else est = away[j] * prod; /* product of the growth of columns 0..j-1 */
                prod *= gfj;
                if (!isfinite(est) || !isfinite(pivj)) nonfinite = 1;
                double ap = alpha * pivj;
                if (!(ap >= est)) lu = 0;
                double den = ap > est ? ap : est;
                if (den < DBL_MIN) den = DBL_MIN;
                double r = (ap - est) / den;
                if (r < margin) margin = r;
                if (pivj < smin) smin = pivj;
                if (est > emax) emax = est;
            }
            if (nonfinite) { lu = 0; margin = -1.0; }
            s = smin; m = emax;
        } else { /* CRIT_RANDOM: LU with probability alpha/100 */
            double u = oracle_uniform(seed, (uint64_t)k);
            lu = (u < alpha / 100.0);
            margin = alpha / 100.0 - u;
        }
        if (nonfinite && diag) diag[DG_NONFINITE] = 1.0;
        if (dec) dec[k] = (int8_t)lu;
        if (s_out) s_out[k] = s;
        if (m_out) m_out[k] = m;
        if (margin_out) margin_out[k] = margin;

        if (lu) {
            if (zero_piv && diag && diag[DG_INFO] == 0.0) diag[DG_INFO] = (double)(k * nb + zero_piv);
            if (a2) {
                /* ---- LU step, variant A2 (Sec. 2.3): Eliminate A_ik <- A_ik U_kk^{-1}
                 * with U_kk the R factor in A_kk, Apply A_kj <- Q_kk^T A_kj (ORMQR) */
                if (ipiv) for (int64_t c = 0; c < mk; ++c) ipiv[k * nb + c] = (int32_t)c;
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t t = 0; t < 2 * (n - k - 1); ++t) {
                    if (t < n - k - 1) {
                        int64_t i = k + 1 + t;
                        trsm_right_upper(mk, Akk, lda, tsize(N, nb, i), &A[IX(i * nb, k * nb, lda)], lda);
                    } else {
                        int64_t j = k + 1 + (t - (n - k - 1));
                        oracle_unmqr(mk, Akk, lda, Tkk, nb, tsize(N, nb, j), &A[IX(k * nb, j * nb, lda)], lda);
                    }
                }
                if (B) oracle_unmqr(mk, Akk, lda, Tkk, nb, nrhs, &B[IX(k * nb, 0, ldb)], ldb);
            } else {
                /* ---- LU step, variant A1 (Alg. 2) */
                for (int64_t j = 0; j < mk; ++j)
                    for (int64_t i = 0; i < mk; ++i) Akk[IX(i, j, lda)] = W[IX(i, j, nb)];
                if (ipiv) for (int64_t c = 0; c < mk; ++c) ipiv[k * nb + c] = d == 1 ? piv[c] : dpiv[c];
                if (d > 1) {
                    /* the domain's interchanges on the trailing columns of its rows
                     * (and on B), and its multipliers below the diagonal tile; the
                     * diagonal tile then needs no further pivoting (piv = identity) */
                    domain_swap(mk, dpiv, dtile, nb, A, lda, (k + 1) * nb, N);
                    if (B) domain_swap(mk, dpiv, dtile, nb, B, ldb, 0, nrhs);
                    for (int64_t t = 1; t < d; ++t)
                        for (int64_t j = 0; j < mk; ++j)
                            for (int64_t r = 0; r < tsize(N, nb, dtile[t]); ++r)
                                A[IX(dtile[t] * nb + r, k * nb + j, lda)] = Wd[IX(t * nb + r, j, R)];
                }
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t t = 0; t < 2 * (n - k - 1); ++t) {
                    if (t < n - k - 1) { /* Eliminate A_ik (done by the domain factorization for its tiles) */
                        int64_t i = k + 1 + t;
                        int in_domain = 0;
                        for (int64_t q = 1; q < d; ++q) in_domain |= dtile[q] == i;
                        if (!in_domain) trsm_right_upper(mk, W, nb, tsize(N, nb, i), &A[IX(i * nb, k * nb, lda)], lda);
                    } else { /* Apply A_kj */
                        int64_t j = k + 1 + (t - (n - k - 1));
                        swptrsm(mk, W, nb, piv, tsize(N, nb, j), &A[IX(k * nb, j * nb, lda)], lda);
                    }
                }
                if (B) swptrsm(mk, W, nb, piv, nrhs, &B[IX(k * nb, 0, ldb)], ldb);
            }
            /* ---- Update (both variants) */
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
            for (int64_t j = k + 1; j < n; ++j)
                for (int64_t i = k + 1; i < n; ++i)
                    gemm_minus(tsize(N, nb, i), tsize(N, nb, j), mk, &A[IX(i * nb, k * nb, lda)], lda,
                               &A[IX(k * nb, j * nb, lda)], lda, &A[IX(i * nb, j * nb, lda)], lda);
            if (B)
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t i = k + 1; i < n; ++i)
                    gemm_minus(tsize(N, nb, i), nrhs, mk, &A[IX(i * nb, k * nb, lda)], lda,
                               &B[IX(k * nb, 0, ldb)], ldb, &B[IX(i * nb, 0, ldb)], ldb);
            if (diag) {
                diag[DG_NLU] += 1.0;
                /* per-step growth inequalities of Sec. 3.1 and 3.2 */
                for (int64_t j = k + 1; j < n; ++j) {
                    double colb = 0.0, cola = 0.0;
                    double akj = nrm_before[IX(k, j, n)];
                    for (int64_t i = k + 1; i < n; ++i) {
                        double after = oracle_tile_norm1(&A[IX(i * nb, j * nb, lda)], lda, tsize(N, nb, i), tsize(N, nb, j));
                        double rhs = nrm_before[IX(i, j, n)] + alpha * akj;
                        double ratio = rhs > 0 ? after / rhs : (after > 0 ? INFINITY : 0.0);
                        if (ratio > diag[DG_MAXINEQ]) diag[DG_MAXINEQ] = ratio;
                        colb += nrm_before[IX(i, j, n)];
                        cola += after;
                    }
                    double rhs = colb + alpha * akj;
                    double ratio = rhs > 0 ? cola / rhs : (cola > 0 ? INFINITY : 0.0);
                    if (ratio > diag[DG_SUMINEQ]) diag[DG_SUMINEQ] = ratio;
                }
            }
        } else {
            /* ---- QR step with TS kernels, flat tree: eliminator of every A_ik is A_kk (Alg. 3, 4a).
             * A1: A_kk was never modified (the LU attempt ran on the copy W: restore
             * is a no-op).  A2: the GEQRT of A_kk is the Factor's, kept (Sec. 2.3). */
            if (ipiv) for (int64_t c = 0; c < mk; ++c) ipiv[k * nb + c] = (int32_t)c;
            /* the elimination list of Alg. 3: within each group its head
             * eliminates the other tiles with TS kernels (Alg. 4a); with one
             * group (qr_tree = 0) the head is A_kk and this is the flat tree */
            const int64_t G = qr_groups(k, n, qr_tree, ghead);
            for (int64_t g = 0; g < G; ++g) {
                const int64_t h = ghead[g];
                double *Ah = &A[IX(h * nb, k * nb, lda)];
                double *Th = (Tq && h != k) ? &Tq[((size_t)k * n + h) * nb * nb] : Tkk;
                if (!(a2 && h == k)) oracle_geqrt(mk, Ah, lda, Th, nb);
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t j = k + 1; j < n; ++j)
                    oracle_unmqr(mk, Ah, lda, Th, nb, tsize(N, nb, j), &A[IX(h * nb, j * nb, lda)], lda);
                if (B) oracle_unmqr(mk, Ah, lda, Th, nb, nrhs, &B[IX(h * nb, 0, ldb)], ldb);
                for (int64_t i = h + 1; i < ghead[g + 1]; ++i) {
                    int64_t mi = tsize(N, nb, i);
                    double *Aik = &A[IX(i * nb, k * nb, lda)];
                    double *Tik = Tq ? &Tq[((size_t)k * n + i) * nb * nb] : Tloc;
                    oracle_tsqrt(mk, Ah, lda, mi, Aik, lda, Tik, nb);
#pragma omp parallel for schedule(dynamic, 1)
                    for (int64_t j = k + 1; j < n; ++j)
                        oracle_tsmqr(mk, mi, Aik, lda, Tik, nb, tsize(N, nb, j),
                                     &A[IX(h * nb, j * nb, lda)], lda, &A[IX(i * nb, j * nb, lda)], lda);
                    if (B)
                        oracle_tsmqr(mk, mi, Aik, lda, Tik, nb, nrhs, &B[IX(h * nb, 0, ldb)], ldb,
                                     &B[IX(i * nb, 0, ldb)], ldb);
                }
            }
            /* the heads by a binary tree of TT kernels (Alg. 4b) */
            for (int64_t dd = 1; dd < G; dd *= 2)
                for (int64_t g = 0; g + dd < G; g += 2 * dd) {
                    const int64_t h0 = ghead[g], h1 = ghead[g + dd];
                    double *A0 = &A[IX(h0 * nb, k * nb, lda)], *A1 = &A[IX(h1 * nb, k * nb, lda)];
                    double *T1 = &Tt[((size_t)k * n + h1) * nb * nb];
                    oracle_ttqrt(mk, A0, lda, A1, lda, T1, nb);
#pragma omp parallel for schedule(dynamic, 1)
                    for (int64_t j = k + 1; j < n; ++j)
                        oracle_ttmqr(mk, A1, lda, T1, nb, tsize(N, nb, j), &A[IX(h0 * nb, j * nb, lda)], lda,
                                     &A[IX(h1 * nb, j * nb, lda)], lda);
                    if (B)
                        oracle_ttmqr(mk, A1, lda, T1, nb, nrhs, &B[IX(h0 * nb, 0, ldb)], ldb,
                                     &B[IX(h1 * nb, 0, ldb)], ldb);
                }
        }
        if (diag) diag[DG_TRUEFLOPS] += step_units_v(n - k - 1, !lu, a2) * (double)nb * (double)nb * (double)nb;
    }
    if (diag) {
        diag[DG_GROWTH_TILE] = max_tile0 > 0 ? max_tile / max_tile0 : 0.0;
        diag[DG_GROWTH_ELEM] = max_elem0 > 0 ? max_elem / max_elem0 : 0.0;
    }
    free(piv); free(W); free(Tloc); free(colsum_scratch); free(away); free(lmax); free(nrm_before);
    free(dtile); free(Wd); free(Pd); free(dpiv); free(ghead);
    return 0;
}

int oracle_factor_ex(int64_t N, double *A, int64_t lda, int64_t nb, int32_t criterion, double alpha,
                     uint64_t seed, const int8_t *forced, int32_t mumps_reading, int64_t nsteps,
                     double *B, int64_t ldb, int64_t nrhs,
                     int32_t *ipiv, double *Tq, int8_t *dec, double *s_out, double *m_out,
                     double *margin_out, double *diag, int32_t domain_stride, int32_t invnorm_estimate,
                     int32_t lu_variant)
{
    return oracle_factor_t(N, A, lda, nb, criterion, alpha, seed, forced, mumps_reading, nsteps, B, ldb, nrhs,
                           ipiv, Tq, dec, s_out, m_out, margin_out, diag, domain_stride, invnorm_estimate,
                           lu_variant, 0, NULL);
}

int oracle_factor_domain(int64_t N, double *A, int64_t lda, int64_t nb, int32_t criterion, double alpha,
                         uint64_t seed, const int8_t *forced, int32_t mumps_reading, int64_t nsteps,
                         double *B, int64_t ldb, int64_t nrhs,
                         int32_t *ipiv, double *Tq, int8_t *dec, double *s_out, double *m_out,
                         double *margin_out, double *diag, int32_t domain_stride)
{
    return oracle_factor_ex(N, A, lda, nb, criterion, alpha, seed, forced, mumps_reading, nsteps, B, ldb, nrhs,
                            ipiv, Tq, dec, s_out, m_out, margin_out, diag, domain_stride, 0, 1);
}

int oracle_factor(int64_t N, double *A, int64_t lda, int64_t nb, int32_t criterion, double alpha,
                  uint64_t seed, const int8_t *forced, int32_t mumps_reading, int64_t nsteps,
                  double *B, int64_t ldb, int64_t nrhs,
                  int32_t *ipiv, double *Tq, int8_t *dec, double *s_out, double *m_out,
                  double *margin_out, double *diag)
{
    return oracle_factor_domain(N, A, lda, nb, criterion, alpha, seed, forced, mumps_reading, nsteps, B, ldb, nrhs,
                                ipiv, Tq, dec, s_out, m_out, margin_out, diag, 0);
}

/* ---------------------------------------------------------------------- */
/* Second-pass solve (Sec. 2.4): replay the stored transformations on B,    */
/* then block back-substitution with the upper-triangular factor.  F, ipiv, */
/* Tq, dec are oracle_factor outputs of a full factorization.              */
/* ---------------------------------------------------------------------- */
/* lu_variant 2: an LU step replays Q_kk^T (from V_kk and Tq(k,k)) on B_k
 * before the block eliminations below it (Sec. 2.3).  qr_tree, Tt: a QR step
 * replays its elimination tree (qr_groups) in the factorization's order. */
void oracle_forward_t(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                      const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                      int32_t domain_stride, int32_t lu_variant, int32_t qr_tree, const double *Tt)
{
    const int64_t n = (N + nb - 1) / nb;
    int64_t *dtile = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *ident = (int32_t *)malloc((size_t)nb * sizeof(int32_t));
    int64_t *ghead = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    for (int64_t c = 0; c < nb; ++c) ident[c] = (int32_t)c;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t mk = tsize(N, nb, k);
        const double *Fkk = &F[IX(k * nb, k * nb, ldf)];
        double *Bk = &B[IX(k * nb, 0, ldb)];
        const int64_t d = domain_tiles(k, n, domain_stride, dtile);
        if (dec[k] && lu_variant == 2) {
            oracle_unmqr(mk, Fkk, ldf, &Tq[((size_t)k * n + k) * nb * nb], nb, nrhs, Bk, ldb);
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t i = k + 1; i < n; ++i)
                gemm_minus(tsize(N, nb, i), nrhs, mk, &F[IX(i * nb, k * nb, ldf)], ldf, Bk, ldb,
                           &B[IX(i * nb, 0, ldb)], ldb);
        } else if (dec[k] && d > 1) {
            domain_swap(mk, &ipiv[k * nb], dtile, nb, B, ldb, 0, nrhs);
            swptrsm(mk, Fkk, ldf, ident, nrhs, Bk, ldb);
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t i = k + 1; i < n; ++i)
                gemm_minus(tsize(N, nb, i), nrhs, mk, &F[IX(i * nb, k * nb, ldf)], ldf, Bk, ldb,
                           &B[IX(i * nb, 0, ldb)], ldb);
        } else if (dec[k]) {
            swptrsm(mk, Fkk, ldf, &ipiv[k * nb], nrhs, Bk, ldb);
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t i = k + 1; i < n; ++i)
                gemm_minus(tsize(N, nb, i), nrhs, mk, &F[IX(i * nb, k * nb, ldf)], ldf, Bk, ldb,
                           &B[IX(i * nb, 0, ldb)], ldb);
        } else {
            const int64_t G = qr_groups(k, n, qr_tree, ghead);
            for (int64_t g = 0; g < G; ++g) {
                const int64_t h = ghead[g];
                const double *Fh = &F[IX(h * nb, k * nb, ldf)];
                double *Bh = &B[IX(h * nb, 0, ldb)];
                oracle_unmqr(mk, Fh, ldf, &Tq[((size_t)k * n + h) * nb * nb], nb, nrhs, Bh, ldb);
                for (int64_t i = h + 1; i < ghead[g + 1]; ++i)
                    oracle_tsmqr(mk, tsize(N, nb, i), &F[IX(i * nb, k * nb, ldf)], ldf,
                                 &Tq[((size_t)k * n + i) * nb * nb], nb, nrhs, Bh, ldb, &B[IX(i * nb, 0, ldb)], ldb);
            }
            for (int64_t dd = 1; dd < G; dd *= 2)
                for (int64_t g = 0; g + dd < G; g += 2 * dd) {
                    const int64_t h0 = ghead[g], h1 = ghead[g + dd];
                    oracle_ttmqr(mk, &F[IX(h1 * nb, k * nb, ldf)], ldf, &Tt[((size_t)k * n + h1) * nb * nb], nb, nrhs,
                                 &B[IX(h0 * nb, 0, ldb)], ldb, &B[IX(h1 * nb, 0, ldb)], ldb);
                }
        }
    }
    free(dtile); free(ident); free(ghead);
}

void oracle_forward_v(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                      const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                      int32_t domain_stride, int32_t lu_variant)
{
    oracle_forward_t(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, domain_stride, lu_variant, 0, NULL);
}

void oracle_forward_domain(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                           const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                           int32_t domain_stride)
{
    oracle_forward_v(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, domain_stride, 1);
}

void oracle_forward(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                    const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs)
{
    oracle_forward_domain(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, 0);
}

void oracle_backward(int64_t N, const double *F, int64_t ldf, int64_t nb, double *B, int64_t ldb, int64_t nrhs)
{
    const int64_t n = (N + nb - 1) / nb;
    for (int64_t k = n - 1; k >= 0; --k) {
        const int64_t mk = tsize(N, nb, k);
        double *Bk = &B[IX(k * nb, 0, ldb)];
        for (int64_t j = k + 1; j < n; ++j)
            gemm_minus(mk, nrhs, tsize(N, nb, j), &F[IX(k * nb, j * nb, ldf)], ldf, &B[IX(j * nb, 0, ldb)], ldb, Bk, ldb);
        const double *U = &F[IX(k * nb, k * nb, ldf)];
        for (int64_t q = 0; q < nrhs; ++q)
            for (int64_t c = mk - 1; c >= 0; --c) {
                double x = Bk[IX(c, q, ldb)] / U[IX(c, c, ldf)];
                Bk[IX(c, q, ldb)] = x;
                for (int64_t r = 0; r < c; ++r) Bk[IX(r, q, ldb)] -= U[IX(r, c, ldf)] * x;
            }
    }
}

void oracle_solve(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                  const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs)
{
    oracle_forward(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs);
    oracle_backward(N, F, ldf, nb, B, ldb, nrhs);
}

void oracle_solve_domain(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                         const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                         int32_t domain_stride)
{
    oracle_forward_domain(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, domain_stride);
    oracle_backward(N, F, ldf, nb, B, ldb, nrhs);
}

void oracle_solve_v(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                    const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                    int32_t domain_stride, int32_t lu_variant)
{
    oracle_forward_v(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, domain_stride, lu_variant);
    oracle_backward(N, F, ldf, nb, B, ldb, nrhs);
}

void oracle_solve_t(int64_t N, const double *F, int64_t ldf, int64_t nb, const int32_t *ipiv,
                    const double *Tq, const int8_t *dec, double *B, int64_t ldb, int64_t nrhs,
                    int32_t domain_stride, int32_t lu_variant, int32_t qr_tree, const double *Tt)
{
    oracle_forward_t(N, F, ldf, nb, ipiv, Tq, dec, B, ldb, nrhs, domain_stride, lu_variant, qr_tree, Tt);
    oracle_backward(N, F, ldf, nb, B, ldb, nrhs);
}

/* Table 1 flop count of a decision sequence (flops). */
double oracle_true_flops(int64_t N, int64_t nb, const int8_t *dec)
{
    const int64_t n = (N + nb - 1) / nb;
    double f = 0.0;
    for (int64_t k = 0; k < n; ++k) f += step_units(n - k - 1, !dec[k]);
    return f * (double)nb * (double)nb * (double)nb;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
