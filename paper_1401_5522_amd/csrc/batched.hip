// Many independent systems A_s x_s = b_s of uneven size in one persistent
// launch.  Each workgroup takes systems from a queue (largest first) and runs
// the whole hybrid LU-QR of Alg. 1 on one system by itself: per step the
// GETRF copy, the exact inverse norm and the Max or Sum test of Sec. 3, then
// an LU step (Alg. 2) or a flat-tree QR step (Alg. 3/4a), all on FP32 tiles
// with MFMA contractions, and finally the solve of Sec. 2.4 with FP64
// iterative refinement against the caller's FP64 matrix.  Tile sizes 32 and
// 64; the same readings of the paper as the single-system path (identity
// padding of the last tile, first-max pivoting, zero pivot => QR, ties => LU).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "engine.h"

namespace lq {

// ---------------------------------------------------------------------------
// Per-system workspace (byte offsets from the system's base), all 256-byte
// aligned.  Tiles are nb x nb column-major, tile (i,j) at (j*n + i)*nb^2.
// ---------------------------------------------------------------------------
struct BLayout {
    int64_t At, Tf, Li, Di, perm, y, z, x, r, d, total;
};
LQ_HD BLayout blayout(int64_t N, int nb) {
    const int64_t n = (N + nb - 1) / nb, Np = n * nb, t2 = (int64_t)nb * nb;
    BLayout L;
    int64_t o = 0;
    auto take = [&](int64_t b) { int64_t r = o; o = (int64_t)align256((size_t)(o + b)); return r; };
    L.At = take(n * n * t2 * 4);
    L.Tf = take(n * n * t2 * 4);
    L.Li = take(n * t2 * 8);
    L.Di = take(n * t2 * 8);
    L.perm = take(n * nb * 4);
    L.y = take(Np * 8);
    L.z = take(Np * 8);
    L.x = take(Np * 8);
    L.r = take(Np * 8);
    L.d = take(Np * 8);
    L.total = o;
    return L;
}

struct BSys {
    int64_t off;  // byte offset of the system's workspace
    int N, nb, lda, ldb, ldx, idx;
};

struct BArgs {
    const BSys *sys;  // in queue order (largest first)
    int batch;
    int *counter;
    char *ws;
    const double *const *A;
    const double *const *B;
    double *const *X;
    int crit;
    double alpha;
    int max_iter;
    int8_t *dec;
    int dec_stride;
    double *eta;
    int *iters;
};

// ---- LDS plan (bytes), shared by both tile sizes --------------------------
constexpr int B_NBMAX = 64;
constexpr int B_W = 0;                                   // FP64 GETRF copy
constexpr int B_UI = B_W + B_NBMAX * B_NBMAX * 8;        // FP64 U^-1 or R^-1
constexpr int B_LI = B_UI + B_NBMAX * B_NBMAX * 8;       // FP64 L^-1
constexpr int B_MMA = B_LI + B_NBMAX * B_NBMAX * 8;      // wg_mma staging
constexpr int B_QR = B_MMA + 9216;                       // Ys, Ts, Rb, PanelLds
constexpr int B_VEC = B_QR + 20480;                      // vectors of the solve
constexpr int B_RED = B_VEC + 4 * B_NBMAX * 8;           // reductions
constexpr int B_LDS = B_RED + WG * 8 + 64;

static_assert(mma_lds_bytes<P32, 64, 64, 16>() <= 9216, "mma staging fits");
static_assert(qr_vblk<64>() * 4 + 2 * IB * IB * 4 + (int)sizeof(PanelLds) <= 20480, "QR staging fits");
static_assert(qr_lds<64, P32>() <= 20480, "QR staging fits");

LQ_DEV double block_max(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        double m = red[threadIdx.x];
        for (int t = threadIdx.x + 64; t < WG; t += 64) m = nmax(m, red[t]);
        m = wave_max(m);
        if (threadIdx.x == 0) red[WG] = m;
    }
    __syncthreads();
    const double r = red[WG];
    __syncthreads();
    return r;
}
LQ_DEV double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        double m = 0.0;
        for (int t = threadIdx.x; t < WG; t += 64) m += red[t];
        m = wave_sum(m);
        if (threadIdx.x == 0) red[WG] = m;
    }
    __syncthreads();
    const double r = red[WG];
    __syncthreads();
    return r;
}

// GEPP on the FP64 copy W (LDS, column-major NB x NB): first-max pivot per
// column, a column with an exactly zero pivot is skipped (returns its 1-based
// index as the first zero pivot).  perm[r] = original local row of row r.
template <int NB>
LQ_DEV int b_getrf(double *W, int *perm, int *ipiv_lds) {
    const int tid = threadIdx.x;
    __shared__ int piv_s, zp_s;
    if (tid == 0) zp_s = 0;
    for (int r = tid; r < NB; r += WG) perm[r] = r;
    __syncthreads();
    for (int c = 0; c < NB; ++c) {
        if (tid < 64) {
            const int r = c + tid;
            double v = r < NB ? fabs(W[r + c * NB]) : -1.0;
            int idx = r < NB ? r : NB;
            wave_argmax(v, idx);
            if (tid == 0) {
                if (idx >= NB) idx = c;  // all candidates NaN: keep the diagonal
                piv_s = idx;
                if (W[idx + c * NB] == 0.0 && zp_s == 0) zp_s = c + 1;
            }
        }
        __syncthreads();
        const int p = piv_s;
        if (p != c) {
            for (int q = tid; q < NB; q += WG) {
                const double t = W[c + q * NB];
                W[c + q * NB] = W[p + q * NB];
                W[p + q * NB] = t;
            }
            if (tid == 0) { const int t = perm[c]; perm[c] = perm[p]; perm[p] = t; }
        }
        if (tid == 0) ipiv_lds[c] = p;
        __syncthreads();
        const double pv = W[c + c * NB];
        if (pv != 0.0) {
            for (int r = c + 1 + tid; r < NB; r += WG) W[r + c * NB] /= pv;
            __syncthreads();
            for (int e = tid; e < (NB - c - 1) * (NB - c - 1); e += WG) {
                const int r = c + 1 + e % (NB - c - 1), q = c + 1 + e / (NB - c - 1);
                W[r + q * NB] -= W[r + c * NB] * W[c + q * NB];
            }
        }
        __syncthreads();
    }
    return zp_s;
}

// Column j of U^-1 (upper, non-unit) and of L^-1 (unit lower) by thread j,
// from the factored W; all in FP64 LDS.  Src(r, c) reads the factors.
template <int NB, class Src>
LQ_DEV void b_trinv(Src src, double *Ui, double *Li, bool lower) {
    const int j = threadIdx.x;
    if (j < NB) {
        for (int r = 0; r < NB; ++r) Ui[r + j * NB] = 0.0;
        for (int r = j; r >= 0; --r) {
            double acc = r == j ? 1.0 : 0.0;
            for (int c = r + 1; c <= j; ++c) acc -= src(r, c) * Ui[c + j * NB];
            Ui[r + j * NB] = acc / src(r, r);
        }
        if (lower) {
            for (int r = 0; r < NB; ++r) Li[r + j * NB] = r == j ? 1.0 : 0.0;
            for (int r = j + 1; r < NB; ++r) {
                double acc = 0.0;
                for (int c = j; c < r; ++c) acc -= src(r, c) * Li[c + j * NB];
                Li[r + j * NB] = acc;
            }
        }
    }
    __syncthreads();
}

template <int NB>
LQ_DEV float *btile(float *At, int n, int i, int j) { return At + ((size_t)j * n + i) * NB * NB; }

// ---------------------------------------------------------------------------
// One system.
// ---------------------------------------------------------------------------
template <int NB>
LQ_DEV void bsys_factor(const BArgs &a, const BSys &S, char *lds, int8_t *dec_out, int *dec_lds) {
    const int tid = threadIdx.x;
    const int N = S.N, n = (N + NB - 1) / NB, Np = n * NB;
    const BLayout L = blayout(N, NB);
    char *w = a.ws + S.off;
    float *At = (float *)(w + L.At);
    float *Tf = (float *)(w + L.Tf);
    double *LiG = (double *)(w + L.Li);
    double *DiG = (double *)(w + L.Di);
    int *permG = (int *)(w + L.perm);
    double *W = (double *)(lds + B_W);
    double *Ui = (double *)(lds + B_UI);
    double *Li = (double *)(lds + B_LI);
    char *msm = lds + B_MMA;
    double *red = (double *)(lds + B_RED);
    float *Ys = (float *)(lds + B_QR);
    float *Ts = Ys + qr_vblk<NB>();
    float *Rb = Ts + IB * IB;
    PanelLds *pl = (PanelLds *)(Rb + IB * IB);
    __shared__ int perm_l[B_NBMAX], ipiv_l[B_NBMAX];
    const double *A = a.A[S.idx];
    // tile-major FP32 copy with identity padding
    for (int64_t e = tid; e < (int64_t)Np * Np; e += WG) {
        const int64_t t = e / (NB * NB), ee = e % (NB * NB);
        const int i = (int)(t % n), j = (int)(t / n);
        const int r = i * NB + (int)(ee % NB), c = j * NB + (int)(ee / NB);
        At[e] = (r < N && c < N) ? (float)A[r + (int64_t)c * S.lda] : (r == c ? 1.0f : 0.0f);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int rest = n - k - 1;
        const int mk = k < n - 1 ? NB : N - (n - 1) * NB;
        float *Akk = btile<NB>(At, n, k, k);
        // -- GETRF on the FP64 copy, exact inverse norm over the real columns
        for (int e = tid; e < NB * NB; e += WG) W[e] = (double)Akk[e];
        __syncthreads();
        const int zp = b_getrf<NB>(W, perm_l, ipiv_l);
        double s = 0.0;
        if (!zp) {
            b_trinv<NB>([&](int r, int c) { return W[r + c * NB]; }, Ui, Li, true);
            double cs = 0.0;
            if (tid < mk) {  // column tid of U^-1 L^-1
                for (int r = 0; r < NB; ++r) {
                    double acc = 0.0;
                    for (int c = r; c < NB; ++c) acc += Ui[r + c * NB] * Li[c + tid * NB];
                    cs += fabs(acc);
                }
            }
            s = 1.0 / block_max(cs, red);
        }
        // -- sub-diagonal tile norms ||A_ik||_1 (max or sum)
        double m = 0.0;
        for (int i = k + 1; i < n; ++i) {
            const float *T = btile<NB>(At, n, i, k);
            double cs = 0.0;
            if (tid < NB)
                for (int r = 0; r < NB; ++r) cs += fabs((double)T[r + tid * NB]);
            const double tn = block_max(cs, red);
            m = a.crit == LUQR_CRIT_SUM ? m + tn : nmax(m, tn);
        }
        int lu;
        if (isinf(a.alpha)) lu = 1;
        else if (a.alpha == 0.0 || zp) lu = 0;
        else if (!(isfinite(s) && isfinite(m))) lu = 0;
        else lu = a.alpha * s >= m;
        if (tid == 0) {
            dec_lds[k] = lu;
            if (dec_out) dec_out[k] = (int8_t)lu;
        }
        if (lu) {
            // zero pivot with alpha = inf: continue as LAPACK does (U^-1 from the zero diagonal is inf)
            if (zp) b_trinv<NB>([&](int r, int c) { return W[r + c * NB]; }, Ui, Li, true);
            for (int e = tid; e < NB * NB; e += WG) {
                Akk[e] = (float)W[e];
                LiG[(size_t)k * NB * NB + e] = Li[e];
                DiG[(size_t)k * NB * NB + e] = Ui[e];
            }
            for (int r = tid; r < NB; r += WG) permG[k * NB + r] = perm_l[r];
            __syncthreads();
            typedef MmaShape<P32, NB, NB, 2, 2> Sh;
            for (int i = k + 1; i < n; ++i) {  // Eliminate: A_ik <- A_ik U^-1
                float *X = btile<NB>(At, n, i, k);
                typename Tr<P32>::acc acc[Sh::MB][Sh::NBK];
                acc_zero<P32, NB, NB, 2, 2>(acc);
                wg_mma<P32, NB, NB, 2, 2, 16>(
                    acc, NB, [&](int r, int kk) { return (double)X[r + kk * NB]; },
                    [&](int kk, int cc) { return Ui[kk + cc * NB]; }, msm);
                __syncthreads();
                acc_foreach<P32, NB, NB, 2, 2>(acc, [&](int r, int cc, double v) { X[r + cc * NB] = (float)v; });
                __syncthreads();
            }
            for (int j = k + 1; j < n; ++j) {  // Apply: A_kj <- L^-1 P A_kj
                float *X = btile<NB>(At, n, k, j);
                typename Tr<P32>::acc acc[Sh::MB][Sh::NBK];
                acc_zero<P32, NB, NB, 2, 2>(acc);
                wg_mma<P32, NB, NB, 2, 2, 16>(
                    acc, NB, [&](int r, int kk) { return Li[r + kk * NB]; },
                    [&](int kk, int cc) { return (double)X[perm_l[kk] + cc * NB]; }, msm);
                __syncthreads();
                acc_foreach<P32, NB, NB, 2, 2>(acc, [&](int r, int cc, double v) { X[r + cc * NB] = (float)v; });
                __syncthreads();
            }
            for (int j = k + 1; j < n; ++j)  // Update: A_ij -= A_ik A_kj
                for (int i = k + 1; i < n; ++i) {
                    const float *Ai = btile<NB>(At, n, i, k), *Aj = btile<NB>(At, n, k, j);
                    float *C = btile<NB>(At, n, i, j);
                    typename Tr<P32>::acc acc[Sh::MB][Sh::NBK];
                    acc_zero<P32, NB, NB, 2, 2>(acc);
                    wg_mma<P32, NB, NB, 2, 2, 16>(
                        acc, NB, [&](int r, int kk) { return (double)Ai[r + kk * NB]; },
                        [&](int kk, int cc) { return (double)Aj[kk + cc * NB]; }, msm);
                    acc_foreach<P32, NB, NB, 2, 2>(acc, [&](int r, int cc, double v) {
                        C[r + cc * NB] = (float)((double)C[r + cc * NB] - v);
                    });
                    __syncthreads();
                }
            (void)rest;
        } else {
            float *Tkk = btile<NB>(Tf, n, k, k);
            for (int b = 0; b < NB / IB; ++b) {  // GEQRT(A_kk)
                const int c0 = b * IB;
                panel_qr<NB, float, false>(Akk, c0, nullptr, Ys, Ts, pl);
                for (int e = tid; e < IB * IB; e += WG) Tkk[(c0 + e % IB) + (c0 + e / IB) * NB] = Ts[e];
                panel_trailing<NB, P32, false>(Akk, nullptr, b, Ys, Ts);
                __syncthreads();
            }
            const int g = lane_id() >> 4, i16 = lane_id() & 15;
            const int col0 = 16 * wave_id();
            const bool active = col0 < NB;
            for (int j = k + 1; j < n; ++j) {  // UNMQR on A_kj
                float *Akj = btile<NB>(At, n, k, j);
                typename Tr<P32>::acc bot[NB / 16];
                if (active)
                    for (int rb = 0; rb < NB / 16; ++rb)
                        for (int r = 0; r < 4; ++r) bot[rb][r] = Akj[(16 * rb + Tr<P32>::drow(g, r)) + (col0 + i16) * NB];
                for (int b = 0; b < NB / IB; ++b) {
                    __syncthreads();
                    stage_block<NB, float, true>(Akk, Tkk, b * IB, Ys, Ts);
                    __syncthreads();
                    if (active) apply_block<NB, P32, false>(bot, nullptr, b, Ys, Ts);
                }
                if (active)
                    for (int rb = 0; rb < NB / 16; ++rb)
                        for (int r = 0; r < 4; ++r) Akj[(16 * rb + Tr<P32>::drow(g, r)) + (col0 + i16) * NB] = bot[rb][r];
                __syncthreads();
            }
            for (int i = k + 1; i < n; ++i) {
                float *Aik = btile<NB>(At, n, i, k);
                float *Tik = btile<NB>(Tf, n, i, k);
                for (int b = 0; b < NB / IB; ++b) {  // TSQRT(R_kk, A_ik)
                    const int c0 = b * IB;
                    for (int e = tid; e < IB * IB; e += WG) {  // row-major R block
                        const int p = e / IB, q = e % IB;
                        Rb[e] = p <= q ? Akk[(c0 + p) + (c0 + q) * NB] : 0.0f;
                    }
                    __syncthreads();
                    panel_qr<NB, float, true>(Aik, c0, Rb, Ys, Ts, pl);
                    for (int e = tid; e < IB * IB; e += WG) {
                        const int p = e % IB, q = e / IB;
                        if (p <= q) Akk[(c0 + p) + (c0 + q) * NB] = Rb[p * IB + q];
                        Tik[(c0 + p) + (c0 + q) * NB] = Ts[e];
                    }
                    panel_trailing<NB, P32, true>(Aik, Akk, b, Ys, Ts);
                    __syncthreads();
                }
                for (int j = k + 1; j < n; ++j) {  // TSMQR on (A_kj, A_ij)
                    float *Akj = btile<NB>(At, n, k, j), *Aij = btile<NB>(At, n, i, j);
                    float *topc = Akj + (col0 + i16) * NB;
                    typename Tr<P32>::acc bot[NB / 16];
                    if (active)
                        for (int rb = 0; rb < NB / 16; ++rb)
                            for (int r = 0; r < 4; ++r) bot[rb][r] = Aij[(16 * rb + Tr<P32>::drow(g, r)) + (col0 + i16) * NB];
                    for (int b = 0; b < NB / IB; ++b) {
                        __syncthreads();
                        stage_block<NB, float, false>(Aik, Tik, b * IB, Ys, Ts);
                        __syncthreads();
                        if (active) apply_block<NB, P32, true>(bot, topc, b, Ys, Ts);
                    }
                    if (active)
                        for (int rb = 0; rb < NB / 16; ++rb)
                            for (int r = 0; r < 4; ++r) Aij[(16 * rb + Tr<P32>::drow(g, r)) + (col0 + i16) * NB] = bot[rb][r];
                    __syncthreads();
                }
            }
            // R^-1 for the back-substitution, once every TSQRT has updated R_kk
            b_trinv<NB>([&](int r, int c) { return (double)Akk[r + c * NB]; }, Ui, Li, false);
            for (int e = tid; e < NB * NB; e += WG) DiG[(size_t)k * NB * NB + e] = Ui[e];
        }
        __syncthreads();
    }
}

// y <- Q^T-chain and L^-1 replays (forward), then x = back-substitution.
// y, x: FP64 vectors of Np entries in the system's workspace.
template <int NB>
LQ_DEV void bsys_solve1(const BArgs &a, const BSys &S, char *lds, const int *dec_lds, double *y, double *x) {
    const int tid = threadIdx.x;
    const int N = S.N, n = (N + NB - 1) / NB;
    const BLayout L = blayout(N, NB);
    char *w = a.ws + S.off;
    float *At = (float *)(w + L.At);
    float *Tf = (float *)(w + L.Tf);
    const double *LiG = (const double *)(w + L.Li);
    const double *DiG = (const double *)(w + L.Di);
    const int *permG = (const int *)(w + L.perm);
    double *v0 = (double *)(lds + B_VEC);  // NB
    double *v1 = v0 + B_NBMAX;             // NB
    double *wv = v1 + B_NBMAX;             // IB
    for (int k = 0; k < n; ++k) {
        double *yk = y + (size_t)k * NB;
        if (dec_lds[k]) {
            if (tid < NB) v0[tid] = yk[permG[k * NB + tid]];
            __syncthreads();
            if (tid < NB) {
                double acc = 0.0;
                for (int c = 0; c < NB; ++c) acc += LiG[(size_t)k * NB * NB + tid + c * NB] * v0[c];
                yk[tid] = acc;
                v1[tid] = acc;
            }
            __syncthreads();
            for (int i = k + 1; i < n; ++i) {
                const float *Lt = btile<NB>(At, n, i, k);
                if (tid < NB) {
                    double acc = 0.0;
                    for (int c = 0; c < NB; ++c) acc += (double)Lt[tid + c * NB] * v1[c];
                    y[(size_t)i * NB + tid] -= acc;
                }
            }
            __syncthreads();
        } else {
            const float *V = btile<NB>(At, n, k, k);
            const float *T = btile<NB>(Tf, n, k, k);
            if (tid < NB) v0[tid] = yk[tid];
            __syncthreads();
            for (int b = 0; b < NB / IB; ++b) {  // z <- (I - V_b T_b V_b^T)^T z
                const int c0 = b * IB;
                if (tid < IB) {
                    const int q = c0 + tid;
                    double acc = v0[q];
                    for (int r = q + 1; r < NB; ++r) acc += (double)V[r + q * NB] * v0[r];
                    v1[tid] = acc;
                }
                __syncthreads();
                if (tid < IB) {
                    double acc = 0.0;
                    for (int p = 0; p <= tid; ++p) acc += (double)T[(c0 + p) + (c0 + tid) * NB] * v1[p];
                    wv[tid] = acc;
                }
                __syncthreads();
                if (tid >= c0 && tid < NB) {
                    double acc = 0.0;
                    for (int q = 0; q < IB; ++q) {
                        const int qq = c0 + q;
                        const double vv = tid == qq ? 1.0 : (tid > qq ? (double)V[tid + qq * NB] : 0.0);
                        acc += vv * wv[q];
                    }
                    v0[tid] -= acc;
                }
                __syncthreads();
            }
            for (int i = k + 1; i < n; ++i) {
                const float *Y = btile<NB>(At, n, i, k);
                const float *Ti = btile<NB>(Tf, n, i, k);
                double *yi = y + (size_t)i * NB;
                for (int b = 0; b < NB / IB; ++b) {  // [z; y_i] <- Q_b^T [z; y_i], V_b = [E_b; Y_b]
                    const int c0 = b * IB;
                    if (tid < IB) {
                        const int q = c0 + tid;
                        double acc = v0[q];
                        for (int r = 0; r < NB; ++r) acc += (double)Y[r + q * NB] * yi[r];
                        v1[tid] = acc;
                    }
                    __syncthreads();
                    if (tid < IB) {
                        double acc = 0.0;
                        for (int p = 0; p <= tid; ++p) acc += (double)Ti[(c0 + p) + (c0 + tid) * NB] * v1[p];
                        wv[tid] = acc;
                    }
                    __syncthreads();
                    if (tid < IB) v0[c0 + tid] -= wv[tid];
                    if (tid < NB) {
                        double acc = 0.0;
                        for (int q = 0; q < IB; ++q) acc += (double)Y[tid + (c0 + q) * NB] * wv[q];
                        yi[tid] -= acc;
                    }
                    __syncthreads();
                }
            }
            if (tid < NB) yk[tid] = v0[tid];
            __syncthreads();
        }
    }
    for (int k = n - 1; k >= 0; --k) {  // x_k = D_k^-1 y_k; y_i -= U_ik x_k
        if (tid < NB) v0[tid] = y[(size_t)k * NB + tid];
        __syncthreads();
        if (tid < NB) {
            double acc = 0.0;
            for (int c = tid; c < NB; ++c) acc += DiG[(size_t)k * NB * NB + tid + c * NB] * v0[c];
            x[(size_t)k * NB + tid] = acc;
            v1[tid] = acc;
        }
        __syncthreads();
        for (int i = 0; i < k; ++i) {
            const float *U = btile<NB>(At, n, i, k);
            if (tid < NB) {
                double acc = 0.0;
                for (int c = 0; c < NB; ++c) acc += (double)U[tid + c * NB] * v1[c];
                y[(size_t)i * NB + tid] -= acc;
            }
        }
        __syncthreads();
    }
}

template <int NB>
LQ_DEV void bsys_run(const BArgs &a, const BSys &S, char *lds) {
    const int tid = threadIdx.x;
    const int N = S.N, n = (N + NB - 1) / NB, Np = n * NB;
    const BLayout L = blayout(N, NB);
    char *w = a.ws + S.off;
    double *y = (double *)(w + L.y), *x = (double *)(w + L.x), *r = (double *)(w + L.r), *d = (double *)(w + L.d);
    double *red = (double *)(lds + B_RED);
    __shared__ int dec_lds[1024 / 32 + 1];
    bsys_factor<NB>(a, S, lds, a.dec ? a.dec + (size_t)S.idx * a.dec_stride : nullptr, dec_lds);
    const double *A = a.A[S.idx];
    const double *B = a.B[S.idx];
    double *X = a.X[S.idx];
    for (int e = tid; e < Np; e += WG) y[e] = e < N ? B[e] : 0.0;
    __syncthreads();
    bsys_solve1<NB>(a, S, lds, dec_lds, y, x);
    // ||A||_inf once
    double an = 0.0;
    for (int row = tid; row < N; row += WG) {
        double s = 0.0;
        for (int c = 0; c < N; ++c) s += fabs(A[row + (int64_t)c * S.lda]);
        an = fmax(an, s);
    }
    an = block_max(an, red);
    double eta = 0.0;
    int it = 0;
    for (;;) {
        double rn = 0.0, xn = 0.0;
        for (int row = tid; row < N; row += WG) {  // r = b - A x (FP64)
            double s = 0.0;
            for (int c = 0; c < N; ++c) s += A[row + (int64_t)c * S.lda] * x[c];
            const double rr = B[row] - s;
            r[row] = rr;
            rn = fmax(rn, fabs(rr));
            xn = fmax(xn, fabs(x[row]));
        }
        for (int e = N + tid; e < Np; e += WG) r[e] = 0.0;
        rn = block_max(rn, red);
        xn = block_max(xn, red);
        eta = rn / (an * xn);
        if (rn <= (double)N * 1e-16 * an * xn || it >= a.max_iter) break;
        for (int e = tid; e < Np; e += WG) y[e] = r[e];
        __syncthreads();
        bsys_solve1<NB>(a, S, lds, dec_lds, y, d);
        for (int e = tid; e < Np; e += WG) x[e] += d[e];
        __syncthreads();
        ++it;
    }
    for (int e = tid; e < N; e += WG) X[e] = x[e];
    if (tid == 0) {
        if (a.eta) a.eta[S.idx] = eta;
        if (a.iters) a.iters[S.idx] = it;
    }
    __syncthreads();
}

// Persistent kernel: workgroups take systems until the queue is empty.
__global__ __launch_bounds__(WG, 1) void k_batched(BArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[B_LDS];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(a.counter, 1);
        __syncthreads();
        const int t = cur;
        __syncthreads();
        if (t >= a.batch) break;
        const BSys S = a.sys[t];
        if (S.nb == 32) bsys_run<32>(a, S, lds);
        else bsys_run<64>(a, S, lds);
    }
}

static __global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

}  // namespace lq

using namespace lq;

// ---------------------------------------------------------------------------
// Host side: plan, run, autotune.
// ---------------------------------------------------------------------------
struct luqr_batch_s {
    int64_t batch;
    int nmax_tiles;
    BArgs args;
    int grid;
};

static int bhip(hipError_t e) { return e == hipSuccess ? 0 : LUQR_ERR_HIP - (int)e; }

static int64_t plan_layout(int64_t batch, const int64_t *N, const int32_t *nb, int32_t nb_all,
                           std::vector<BSys> *out, int *nmax) {
    int64_t off = 0;
    int nm = 0;
    std::vector<BSys> v((size_t)batch);
    for (int64_t s = 0; s < batch; ++s) {
        const int b = nb ? nb[s] : nb_all;
        if (N[s] < 1 || N[s] > 1024) return -2;
        if (b != 32 && b != 64) return -3;
        v[s].N = (int)N[s];
        v[s].nb = b;
        v[s].idx = (int)s;
        v[s].off = off;
        off += blayout(N[s], b).total;
        nm = std::max(nm, (int)((N[s] + b - 1) / b));
    }
    off = (int64_t)align256((size_t)off);
    const int64_t desc = (int64_t)align256(sizeof(BSys) * (size_t)batch) + 256;  // descriptors + queue counter
    if (out) {
        for (auto &x : v) x.off += desc;
        out->swap(v);
    }
    if (nmax) *nmax = nm;
    return desc + off;
}

extern "C" int64_t luqr_batched_workspace_bytes(int64_t batch, const int64_t *N, const int32_t *nb,
                                                const luqr_opts *o) {
    if (batch < 1) return -1;
    if (!N) return -2;
    if (!o) return -4;
    return plan_layout(batch, N, nb, o->nb, nullptr, nullptr);
}

extern "C" int luqr_batched_plan(int64_t batch, const int64_t *N, const int32_t *nb, const int64_t *lda,
                                 const int64_t *ldb, const int64_t *ldx, const luqr_opts *o, int32_t max_iter,
                                 void *dWork, int64_t work_bytes, luqr_batch *out) {
    if (batch < 1 || batch > (1 << 24)) return -1;
    if (!N) return -2;
    if (!lda || !ldb || !ldx) return -4;
    if (!o) return -7;
    if (max_iter < 0) return -8;
    if (!dWork || ((uintptr_t)dWork & 255)) return -9;
    if (!out) return -11;
    if (o->precision != LUQR_FP32) return LUQR_ERR_UNSUPPORTED;
    if (o->criterion != LUQR_CRIT_MAX && o->criterion != LUQR_CRIT_SUM) return LUQR_ERR_UNSUPPORTED;
    if (o->domain_stride != 0) return LUQR_ERR_UNSUPPORTED;  // each system pivots within its diagonal tiles
    if (o->invnorm_estimate != 0) return LUQR_ERR_UNSUPPORTED;  // the batched kernel takes the exact inverse norm
    if (o->lu_variant == 2) return LUQR_ERR_UNSUPPORTED;  // the batched kernel's LU steps are variant A1
    if (o->qr_tree != 0) return LUQR_ERR_UNSUPPORTED;     // and its QR steps the flat tree
    if (!(o->alpha >= 0.0)) return -7;
    std::vector<BSys> v;
    int nm = 0;
    const int64_t need = plan_layout(batch, N, nb, o->nb, &v, &nm);
    if (need < 0) return (int)need;
    if (work_bytes < need) return -10;
    for (int64_t s = 0; s < batch; ++s) {
        if (lda[s] < N[s] || ldb[s] < N[s] || ldx[s] < N[s]) return -4;
        v[s].lda = (int)lda[s];
        v[s].ldb = (int)ldb[s];
        v[s].ldx = (int)ldx[s];
    }
    // largest first (longest processing time), ties by index
    std::stable_sort(v.begin(), v.end(), [](const BSys &x, const BSys &y) {
        const double cx = (double)x.N * x.N * x.N, cy = (double)y.N * y.N * y.N;
        return cx > cy;
    });
    char *base = (char *)dWork;
    hipError_t e = hipMemcpy(base, v.data(), sizeof(BSys) * (size_t)batch, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(e);
    luqr_batch_s *p = new (std::nothrow) luqr_batch_s;
    if (!p) return LUQR_ERR_HIP - (int)hipErrorOutOfMemory;
    p->batch = batch;
    p->nmax_tiles = nm;
    BArgs &a = p->args;
    a.sys = (const BSys *)base;
    a.batch = (int)batch;
    a.counter = (int *)(base + align256(sizeof(BSys) * (size_t)batch));
    a.ws = base;
    a.crit = o->criterion;
    a.alpha = o->alpha;
    a.max_iter = max_iter;
    a.dec_stride = nm;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    p->grid = (int)std::min<int64_t>(batch, ncu);
    *out = p;
    return 0;
}

extern "C" int luqr_batched_run(luqr_batch p, const double *const *dA, const double *const *dB, double *const *dX,
                                int8_t *dDec, double *dEta, int32_t *dIters, void *stream) {
    if (!p) return -1;
    if (!dA) return -2;
    if (!dB) return -3;
    if (!dX) return -4;
    hipStream_t st = (hipStream_t)stream;
    BArgs a = p->args;
    a.A = dA;
    a.B = dB;
    a.X = dX;
    a.dec = dDec;
    a.eta = dEta;
    a.iters = dIters;
    (void)hipGetLastError();
    k_zero_int<<<1, 64, 0, st>>>(a.counter);
    k_batched<<<p->grid, WG, 0, st>>>(a);
    return bhip(hipGetLastError());
}

extern "C" int luqr_batched_decision_stride(luqr_batch p) { return p ? p->nmax_tiles : -1; }

extern "C" void luqr_batched_destroy(luqr_batch p) { delete p; }

// For each size class [64 * 2^c, 64 * 2^(c+1)) time up to `sample` of its
// systems with n_b = 32 and with n_b = 64 (one persistent launch each, after
// a warm-up launch) and write the faster tile size for every system of the
// class into nb_out.  The systems' own data is used; the outputs of the
// trial runs land in X and are overwritten by the real run.
extern "C" int luqr_batched_autotune(int64_t batch, const int64_t *N, const int64_t *lda, const int64_t *ldb,
                                     const int64_t *ldx, const luqr_opts *o, int32_t max_iter,
                                     const double *const *dA, const double *const *dB, double *const *dX,
                                     int32_t sample, void *dWork, int64_t work_bytes, void *stream,
                                     int32_t *nb_out, float *ms_out) {
    if (batch < 1) return -1;
    if (!N || !lda || !ldb || !ldx || !o || !dA || !dB || !dX || !nb_out) return -2;
    if (sample < 1) return -11;
    hipStream_t st = (hipStream_t)stream;
    const int ncls = 6;
    std::vector<std::vector<int64_t>> cls(ncls);
    for (int64_t s = 0; s < batch; ++s) {
        int c = 0;
        while (c + 1 < ncls && N[s] >= (64LL << (c + 1))) ++c;
        cls[c].push_back(s);
    }
    std::vector<const double *> pa(batch), pb(batch);
    std::vector<double *> px(batch);
    hipError_t e;
    if ((e = hipMemcpy(pa.data(), dA, sizeof(double *) * batch, hipMemcpyDeviceToHost)) != hipSuccess) return bhip(e);
    if ((e = hipMemcpy(pb.data(), dB, sizeof(double *) * batch, hipMemcpyDeviceToHost)) != hipSuccess) return bhip(e);
    if ((e = hipMemcpy(px.data(), dX, sizeof(double *) * batch, hipMemcpyDeviceToHost)) != hipSuccess) return bhip(e);
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return bhip(e);
    if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return bhip(e); }
    int rc = 0;
    for (int c = 0; c < ncls && rc == 0; ++c) {
        if (cls[c].empty()) continue;
        const int64_t m = std::min<int64_t>((int64_t)sample, (int64_t)cls[c].size());
        std::vector<int64_t> sN(m), sl(m), sb(m), sx(m);
        std::vector<const double *> sA(m), sB(m);
        std::vector<double *> sX(m);
        for (int64_t t = 0; t < m; ++t) {
            const int64_t s = cls[c][(size_t)(t * (int64_t)cls[c].size() / m)];
            sN[t] = N[s]; sl[t] = lda[s]; sb[t] = ldb[s]; sx[t] = ldx[s];
            sA[t] = pa[s]; sB[t] = pb[s]; sX[t] = px[s];
        }
        float best = 0.0f;
        int bestnb = 32;
        for (int cand : {32, 64}) {
            luqr_opts oo = *o;
            oo.nb = cand;
            const int64_t need = plan_layout(m, sN.data(), nullptr, cand, nullptr, nullptr);
            const int64_t ptrs = 3 * 8 * m + 256;
            if (need < 0) { rc = (int)need; break; }
            if (need + ptrs > work_bytes) { rc = -13; break; }
            char *pbase = (char *)dWork + ((need + 255) & ~(int64_t)255);
            const double **dA2 = (const double **)pbase;
            const double **dB2 = dA2 + m;
            double **dX2 = (double **)(dB2 + m);
            if ((e = hipMemcpy((void *)dA2, sA.data(), 8 * m, hipMemcpyHostToDevice)) != hipSuccess) { rc = bhip(e); break; }
            if ((e = hipMemcpy((void *)dB2, sB.data(), 8 * m, hipMemcpyHostToDevice)) != hipSuccess) { rc = bhip(e); break; }
            if ((e = hipMemcpy((void *)dX2, sX.data(), 8 * m, hipMemcpyHostToDevice)) != hipSuccess) { rc = bhip(e); break; }
            luqr_batch p = nullptr;
            rc = luqr_batched_plan(m, sN.data(), nullptr, sl.data(), sb.data(), sx.data(), &oo, max_iter, dWork, need, &p);
            if (rc) break;
            rc = luqr_batched_run(p, dA2, dB2, dX2, nullptr, nullptr, nullptr, st);  // warm-up
            if (!rc) (void)hipEventRecord(e0, st);
            if (!rc) rc = luqr_batched_run(p, dA2, dB2, dX2, nullptr, nullptr, nullptr, st);
            if (!rc) (void)hipEventRecord(e1, st);
            if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = bhip(e);
            float ms = 0.0f;
            if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = bhip(e);
            luqr_batched_destroy(p);
            if (rc) break;
            if (ms_out) ms_out[2 * c + (cand == 64)] = ms;
            if (cand == 32 || ms < best) { best = ms; bestnb = cand; }
        }
        for (int64_t s : cls[c]) nb_out[s] = bestnb;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
