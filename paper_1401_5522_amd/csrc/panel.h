// Panel step of the hybrid LU-QR factorization (Alg. 1, Factor + Check):
//   * GETRF with partial pivoting on an FP64 copy of the diagonal tile (the
//     "Backup Panel" / "LU On Panel" tasks of Sec. 4: A_kk itself is left
//     untouched until the decision, so a QR step needs no restore),
//   * the 1-norm of every sub-diagonal tile and the column maxima the MUMPS
//     criterion needs (Sec. 3, Complexity),
//   * the explicit inverses L^{-1}, U^{-1} of the diagonal factors and the
//     exact ||A_kk^{-1}||_1 = max_j ||U^{-1} L^{-1} e_j||_1 (the column
//     permutation P does not change a 1-norm),
//   * the decision itself (Sec. 3.1-3.3 and the random control of Sec. 5.2),
//     written to device memory where the branch kernels read it.
#pragma once
#include <utility>

#include "mma.h"

namespace lq {

// NaN-propagating maximum (a NaN input makes the criterion fail, as in LAPACK's
// treatment of non-finite norms).
LQ_DEV double nmax(double a, double b) { return (b > a || b != b) ? b : a; }
LQ_DEV double wave_nmax(double v) {
    v = nmax(v, xlane<0>(v)); v = nmax(v, xlane<1>(v)); v = nmax(v, xlane<2>(v));
    v = nmax(v, xlane<3>(v)); v = nmax(v, xlane<4>(v)); v = nmax(v, xlane<5>(v));
    return v;
}

// ---------------------------------------------------------------------------
// GETRF of the diagonal tile on its FP64 copy W_k, one workgroup.
// Blocked right-looking LU with partial pivoting: each 32-column panel is
// held in registers, thread t owning tile rows t and t+256, and factored one
// column at a time (column q is its own instantiation, so register indices
// are static): argmax over the workgroup (the first row holding the largest
// magnitude wins ties), exchange of the two rows through LDS, scaling and
// rank-1 update.  The panel's interchanges are then applied to the other
// columns through LDS, U12 = L11^{-1} A12 is solved and A22 -= L21 U12.
// ---------------------------------------------------------------------------
template <int NB> constexpr int lu_rpt() { return NB > 256 ? 2 : 1; }

struct GetrfLds {
    double bv[4];
    int bi[4];
    int dnan;  // the diagonal entry of the column being eliminated is NaN
    int piv[32];
    int zp;
    int tcnt;
    int trow[64], tsrc[64];
    double rowA[32], rowB[32];
};

template <int RPT, int Q>
LQ_DEV void lu_column(double (&P)[RPT][32], int p0, int R, GetrfLds *g) {
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    const int col = p0 + Q;
    double v = -1.0;
    int idx = 0x7fffffff;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {  // rows ascending within the thread
        const int r = tid + 256 * u;
        if (r >= col && r < R) {
            const double a = fabs(P[u][Q]);
            if (a > v) { v = a; idx = r; }
        }
        if (r == col) g->dnan = P[u][Q] != P[u][Q];
    }
    wave_argmax(v, idx);
    if (l == 0) { g->bv[w] = v; g->bi[w] = idx; }
    __syncthreads();  // A
    v = g->bv[0];
    idx = g->bi[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
        const double ov = g->bv[q];
        const int oi = g->bi[q];
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    // The scan that defines the pivot starts at the diagonal and moves to a
    // later row only if its magnitude is strictly larger, so a NaN on the
    // diagonal stays the pivot (and NaNs below it are never chosen); a column
    // of exact zeros below and on the diagonal is skipped (no elimination).
    const bool dnan = g->dnan != 0;
    const bool zero = !dnan && !(v > 0.0);
    const int piv = (zero || dnan) ? col : idx;
    if (tid == 0) {
        g->piv[Q] = piv;
        if (zero && g->zp == 0) g->zp = col + 1;
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = tid + 256 * u;
        if (r == col) {
#pragma unroll
            for (int j = 0; j < 32; ++j) g->rowA[j] = P[u][j];
        }
        if (r == piv) {
#pragma unroll
            for (int j = 0; j < 32; ++j) g->rowB[j] = P[u][j];
        }
    }
    __syncthreads();  // B: rows col and piv exchanged through LDS
    if (!zero) {
        const double pv = g->rowB[Q];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int r = tid + 256 * u;
            if (r == col) {
#pragma unroll
                for (int j = 0; j < 32; ++j) P[u][j] = g->rowB[j];
            } else if (r == piv) {
#pragma unroll
                for (int j = 0; j < 32; ++j) P[u][j] = g->rowA[j];
            }
            if (r > col && r < R) {
                const double lr = P[u][Q] / pv;
                P[u][Q] = lr;
#pragma unroll
                for (int j = Q + 1; j < 32; ++j) P[u][j] -= lr * g->rowB[j];
            }
        }
    }
}

template <int RPT, int... Qs>
LQ_DEV void lu_columns(double (&P)[RPT][32], int p0, int R, GetrfLds *g, std::integer_sequence<int, Qs...>) {
    (lu_column<RPT, Qs>(P, p0, R, g), ...);
}

// The same elimination runs on the diagonal tile alone (R = NB rows, W the
// step's copy, ld NB) or on the stacked diagonal domain (R = d NB rows of the
// tiles k, k+p, ..., W = c.WD, ld DR): the pivot of each column is searched
// over all R rows.  RPT = rows per thread / 256 >= R / 256.
template <int NB, int RPT> struct GetrfSmem {
    static constexpr int BUFN = (NB <= 256 && RPT == 1) ? 32 * (NB + 1) + NB * 33 : 32 * 33;
    double buf[BUFN];  // L21 / U12 staging of the trailing update
    double L11[32 * 33];
    int src[256 * RPT];
    unsigned long long lmx[NB];
    GetrfLds g;
};

template <int NB, class S, int RPT>
LQ_DEV void getrf_core(const Ctx &c, int k, void *smem) {
    const bool dom = c.dcount(k) > 1;
    const int R = dom ? c.dcount(k) * NB : NB;
    const int ldw = dom ? c.DR : NB;
    GetrfSmem<NB, RPT> &sm = *(GetrfSmem<NB, RPT> *)smem;
    double *buf = sm.buf, *L11 = sm.L11;
    int *src = sm.src;
    unsigned long long *lmx = sm.lmx;
    GetrfLds &g = sm.g;
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    double *W = dom ? c.WD : c.W + (size_t)k * NB * NB;
    const S *A = (const S *)c.At + c.toff(k, k);
    for (int e = tid; e < NB; e += WG) lmx[e] = 0ull;
    if (tid == 0) g.zp = 0;
    __syncthreads();
    if (dom) {
        // stacked copy of the domain's tiles and its column maxima (MUMPS
        // local_max over the domain): wave w takes columns w, w+4, ...
        for (int col = w; col < NB; col += 4) {
            double m = 0.0;
            for (int r = l; r < R; r += 64) {
                const S *T = (const S *)c.At + c.toff(k + (int64_t)(r / NB) * c.dstride, k);
                const double a = (double)T[r % NB + (size_t)col * NB];
                W[r + (size_t)col * ldw] = a;
                m = nmax(m, fabs(a));
            }
            m = wave_nmax(m);
            if (l == 0) lmx[col] = (unsigned long long)__double_as_longlong(m);
        }
    } else {
    // copy A_kk -> W (FP64) and its column maxima (MUMPS local_max)
    for (int e0 = 0; e0 < NB * NB; e0 += 8 * WG) {
        double a[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = e0 + t * WG + tid;
            a[t] = e < NB * NB ? (double)A[e] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = e0 + t * WG + tid;
            if (e < NB * NB) W[e] = a[t];
            double m = fabs(a[t]);
            // non-negative doubles (and NaN above them) order as their bit patterns
            if constexpr (NB >= 64) {
                m = wave_nmax(m);  // a wave covers 64 consecutive rows of one column
                if (l == 0 && e < NB * NB) atomicMax(&lmx[e / NB], (unsigned long long)__double_as_longlong(m));
            } else if (e < NB * NB) {  // a wave spans several columns: one atomic per element
                atomicMax(&lmx[e / NB], (unsigned long long)__double_as_longlong(m));
            }
        }
    }
    }
    __syncthreads();
    for (int e = tid; e < NB; e += WG) c.lmax[e] = __longlong_as_double((long long)lmx[e]);
    for (int p0 = 0; p0 < NB; p0 += 32) {
        double P[RPT][32];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int r = tid + 256 * u;
#pragma unroll
            for (int j = 0; j < 32; ++j) P[u][j] = (r >= p0 && r < R) ? W[r + (size_t)(p0 + j) * ldw] : 0.0;
        }
        lu_columns<RPT>(P, p0, R, &g, std::make_integer_sequence<int, 32>{});
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int r = tid + 256 * u;
            if (r >= p0 && r < R) {
#pragma unroll
                for (int j = 0; j < 32; ++j) W[r + (size_t)(p0 + j) * ldw] = P[u][j];
            }
            if (r >= p0 && r < p0 + 32) {
#pragma unroll
                for (int j = 0; j < 32; ++j) L11[j * 33 + (r - p0)] = P[u][j];
            }
        }
        if (tid < 32) c.ipiv[(size_t)k * NB + p0 + tid] = g.piv[tid];
        // rows moved by the panel's interchanges: trow[t] receives row tsrc[t]
        for (int r = p0 + tid; r < R; r += WG) src[r] = r;
        __syncthreads();
        if (tid == 0) {
            for (int q = 0; q < 32; ++q) {
                const int a = p0 + q, b = g.piv[q];
                const int t = src[a]; src[a] = src[b]; src[b] = t;
            }
            int cnt = 0;
            for (int q = 0; q < 32; ++q) {
                const int a = p0 + q, b = g.piv[q];
                if (src[a] != a) { g.trow[cnt] = a; g.tsrc[cnt] = src[a]; src[a] = a; ++cnt; }
                if (b != a && src[b] != b) { g.trow[cnt] = b; g.tsrc[cnt] = src[b]; src[b] = b; ++cnt; }
            }
            g.tcnt = cnt;
        }
        __syncthreads();
        {
            const int cnt = g.tcnt;
            for (int cc = tid; cc < NB; cc += WG) {  // columns outside the panel
                if (cc >= p0 && cc < p0 + 32) continue;
                double v[64];
#pragma unroll
                for (int t = 0; t < 64; ++t) v[t] = t < cnt ? W[g.tsrc[t] + (size_t)cc * ldw] : 0.0;
#pragma unroll
                for (int t = 0; t < 64; ++t)
                    if (t < cnt) W[g.trow[t] + (size_t)cc * ldw] = v[t];
            }
        }
        __syncthreads();
        if (p0 + 32 < NB) {
            for (int cc = p0 + 32 + tid; cc < NB; cc += WG) {  // U12 = L11^{-1} A12
                double x[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) x[q] = W[p0 + q + (size_t)cc * ldw];
#pragma unroll
                for (int q = 0; q < 32; ++q)
#pragma unroll
                    for (int r = q + 1; r < 32; ++r) x[r] -= L11[q * 33 + r] * x[q];
#pragma unroll
                for (int q = 0; q < 32; ++q) W[p0 + q + (size_t)cc * ldw] = x[q];
            }
            __syncthreads();
            if constexpr (NB <= 256 && RPT == 1) {
                // A22 -= L21 U12 on FP64 MFMA: L21 (rows p0+32.., 32 cols) and U12 (32 x
                // trailing cols) staged in LDS, 16x16 output blocks spread over the waves
                constexpr int LDL = NB + 1;
                double *Ls = buf;                 // [32][LDL]
                double *Ub = buf + 32 * LDL;      // [ncol][33]
                const int r0 = p0 + 32, m = NB - r0;
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int r = tid + 256 * u;
                    if (r >= r0 && r < NB) {
#pragma unroll
                        for (int q = 0; q < 32; ++q) Ls[q * LDL + r] = P[u][q];
                    }
                }
                for (int e = tid; e < 32 * m; e += WG) Ub[(e / 32) * 33 + e % 32] = W[p0 + e % 32 + (r0 + e / 32) * NB];
                __syncthreads();
                const int nbk = m / 16;
                const int gq = l >> 4, i16 = l & 15;
                for (int blk = w; blk < nbk * nbk; blk += 4) {
                    const int br = r0 + 16 * (blk % nbk), bc = 16 * (blk / nbk);
                    d4 acc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = W[(br + Tr<P64>::drow(gq, r)) + (r0 + bc + i16) * NB];
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks)
                        acc = Tr<P64>::mma(-Ls[(4 * ks + gq) * LDL + br + i16], Ub[(bc + i16) * 33 + 4 * ks + gq], acc);
#pragma unroll
                    for (int r = 0; r < 4; ++r) W[(br + Tr<P64>::drow(gq, r)) + (r0 + bc + i16) * NB] = acc[r];
                }
                __syncthreads();
            } else {
            constexpr int AW = RPT > 1 ? 16 : 32;  // A22 columns per pass (register budget)
            for (int c0 = p0 + 32; c0 < NB; c0 += AW) {  // A22 -= L21 U12
                for (int e = tid; e < 32 * AW; e += WG)
                    buf[(e / 32) * 33 + e % 32] = W[p0 + e % 32 + (size_t)(c0 + e / 32) * ldw];
                __syncthreads();
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    const int r = tid + 256 * u;
                    if (r < p0 + 32 || r >= R) continue;
                    double wv[AW];
#pragma unroll
                    for (int j = 0; j < AW; ++j) wv[j] = W[r + (size_t)(c0 + j) * ldw];
#pragma unroll
                    for (int q = 0; q < 32; ++q) {
                        const double lq = P[u][q];
#pragma unroll
                        for (int j = 0; j < AW; ++j) wv[j] -= lq * buf[j * 33 + q];
                    }
#pragma unroll
                    for (int j = 0; j < AW; ++j) W[r + (size_t)(c0 + j) * ldw] = wv[j];
                }
                __syncthreads();
            }
            }
        }
        __syncthreads();
    }
    // permutation of the whole tile (or stacked domain): (P A)(r,:) = A(src[r],:)
    for (int r = tid; r < R; r += WG) src[r] = r;
    __syncthreads();
    if (tid == 0) {
        const int *ip = c.ipiv + (size_t)k * NB;
        for (int q = 0; q < NB; ++q) {
            const int p = ip[q];
            const int t = src[q]; src[q] = src[p]; src[p] = t;
        }
        c.zpiv[k] = g.zp;
    }
    __syncthreads();
    if (!dom) {
        for (int r = tid; r < NB; r += WG) c.perm[(size_t)k * NB + r] = src[r];
        return;
    }
    // Domain: the trailing columns of its rows are interchanged before the LU
    // branch's Apply (k_domain_swap), so the diagonal tile's own permutation is
    // the identity; the stacked permutation is kept for that and for the solve.
    // W_k receives the top block L11\U, the diagonal tile after the domain's
    // interchanges (Sec. 3.1), for the inverse norm and the decision.
    for (int r = tid; r < NB; r += WG) c.perm[(size_t)k * NB + r] = r;
    for (int r = tid; r < R; r += WG) c.dperm[(size_t)k * c.DR + r] = src[r];
    double *Wk = c.W + (size_t)k * NB * NB;
    for (int e = tid; e < NB * NB; e += WG) Wk[e] = W[e % NB + (size_t)(e / NB) * ldw];
    // ||A_ik||_1 of the other domain tiles after the interchanges, from the
    // original panel values: row r of tile t is stacked row src[t NB + r]
    double *cs = buf;  // NB column sums
    for (int t = 1; t < R / NB; ++t) {
        const int64_t i = k + (int64_t)t * c.dstride;
        for (int col = w; col < NB; col += 4) {
            double sum = 0.0;
            for (int r = l; r < NB; r += 64) {
                const int so = src[t * NB + r];
                const S *T = (const S *)c.At + c.toff(k + (int64_t)(so / NB) * c.dstride, k);
                sum += fabs((double)T[so % NB + (size_t)col * NB]);
            }
            sum = wave_sum(sum);
            if (l == 0) cs[col] = sum;
        }
        __syncthreads();
        if (tid == 0) {
            double tn = 0.0;
            for (int col = 0; col < NB; ++col) tn = nmax(tn, cs[col]);
            c.tnorm[i] = tn;
        }
        for (int col = tid; col < NB; col += WG) c.away[(size_t)i * NB + col] = 0.0;  // MUMPS: off the domain only
        __syncthreads();
    }
}

// Column sums and column maxima of |A_ik| (one workgroup per tile).
template <int NB, class S>
LQ_DEV void tile_norms(const Ctx &c, int k, int i) {
    __shared__ double cs[NB];
    const int l = lane_id(), w = wave_id();
    const S *A = (const S *)c.At + c.toff(i, k);
    for (int col = w; col < NB; col += 4) {
        double sum = 0.0, mx = 0.0;
        for (int r = l; r < NB; r += 64) {
            double a = fabs((double)A[r + col * NB]);
            sum += a;
            mx = nmax(mx, a);
        }
        sum = wave_sum(sum);
        mx = wave_nmax(mx);
        if (l == 0) { cs[col] = sum; c.away[(size_t)i * NB + col] = mx; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int col = 0; col < NB; ++col) t = nmax(t, cs[col]);
        c.tnorm[i] = t;
    }
}

template <int NB, class S>
__global__ __launch_bounds__(WG) void k_panel_a(Ctx c, int k) {
    constexpr size_t S1 = sizeof(GetrfSmem<NB, 1>), S2 = sizeof(GetrfSmem<NB, 2>);
    __shared__ __attribute__((aligned(16))) char smem[S1 > S2 ? S1 : S2];
    if (blockIdx.x == 0) {
        if constexpr (NB <= 256) {
            if (c.dcount(k) > 1) getrf_core<NB, S, 2>(c, k, smem);  // stacked domain of up to 512 rows
            else getrf_core<NB, S, 1>(c, k, smem);
        } else {
            getrf_core<NB, S, 2>(c, k, smem);
        }
    } else if (!c.indom(k, k + (int)blockIdx.x)) {
        tile_norms<NB, S>(c, k, k + (int)blockIdx.x);  // the domain's tiles are measured after its GEPP
    }
}

// ---------------------------------------------------------------------------
// Explicit inverse of a triangular tile, one wave per column: upper (non-unit,
// back substitution) or unit lower (forward substitution).  32-column blocks
// of the triangle are staged in LDS and shared by the four waves.
// gate: if non-null, run only when *gate == gate_val (device-side decision).
// ---------------------------------------------------------------------------
template <int NB, class SRC>
LQ_DEV void trtri_col(const SRC *M, double *out, bool upper) {
    __shared__ double blk[32 * NB];
    __shared__ double xs[4 * NB];
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    const int j = (int)(blockIdx.x % (NB / 4)) * 4 + w;
    double *x = xs + w * NB;
    for (int r = l; r < NB; r += 64) x[r] = (r == j) ? 1.0 : 0.0;
    wave_sync();
    for (int bi = 0; bi < NB / 32; ++bi) {
        const int cb = upper ? (NB / 32 - 1 - bi) : bi;
        for (int e = tid; e < 32 * NB; e += WG) {
            int r = e % NB, q = e / NB;
            blk[q * NB + r] = (double)M[r + (cb * 32 + q) * NB];
        }
        __syncthreads();
        if (upper) {
            for (int q = 31; q >= 0; --q) {
                const int cc = cb * 32 + q;
                if (cc > j) continue;
                const double xc = x[cc] / blk[q * NB + cc];
                for (int r = l; r < cc; r += 64) x[r] -= blk[q * NB + r] * xc;
                if (l == 0) x[cc] = xc;
                wave_sync();
            }
        } else {
            for (int q = 0; q < 32; ++q) {
                const int cc = cb * 32 + q;
                if (cc < j) continue;
                const double xc = x[cc];
                for (int r = cc + 1 + l; r < NB; r += 64) x[r] -= blk[q * NB + r] * xc;
                wave_sync();
            }
        }
        __syncthreads();
    }
    for (int r = l; r < NB; r += 64) out[r + (size_t)j * NB] = (upper ? r <= j : r >= j) ? x[r] : 0.0;
}

// Panel: grid = NB/2 workgroups; the first NB/4 invert U (into Dinv_k), the
// rest invert L (into Linv_k), both from the GETRF copy W_k.
template <int NB>
__global__ __launch_bounds__(WG) void k_panel_trtri(Ctx c, int k) {
    const double *W = c.W + (size_t)k * NB * NB;
    const bool upper = blockIdx.x < NB / 4;
    trtri_col<NB, double>(W, (upper ? c.Dinv : c.Linv) + (size_t)k * NB * NB, upper);
}

// X = U^{-1} L^{-1} in 64x64 blocks (FP64 MFMA), then partial column sums of
// |X| per row block: invpart[rb*NB + j].
template <int NB>
__global__ __launch_bounds__(WG) void k_panel_invnorm(Ctx c, int k) {
    constexpr int B = NB < 64 ? NB : 64;
    constexpr int NBLK = NB / B;
    __shared__ __attribute__((aligned(16))) char smem[mma_lds_bytes<P64, B, B, 16>()];
    __shared__ double Xs[B * (B + 1)];
    const int rb = blockIdx.x % NBLK, cb = blockIdx.x / NBLK;
    const double *Ui = c.Dinv + (size_t)k * NB * NB;
    const double *Li = c.Linv + (size_t)k * NB * NB;
    typename Tr<P64>::acc acc[B / 2 / 16][B / 2 / 16];
    acc_zero<P64, B, B, 2, 2>(acc);
    wg_mma<P64, B, B, 2, 2, 16>(
        acc, NB, [&](int r, int kk) { return Ui[(rb * B + r) + (size_t)kk * NB]; },
        [&](int kk, int cc) { return Li[kk + (size_t)(cb * B + cc) * NB]; }, smem);
    acc_foreach<P64, B, B, 2, 2>(acc, [&](int r, int cc, double v) { Xs[cc * (B + 1) + r] = fabs(v); });
    __syncthreads();
    for (int cc = threadIdx.x; cc < B; cc += WG) {
        double s = 0.0;
        for (int r = 0; r < B; ++r) s += Xs[cc * (B + 1) + r];
        c.invpart[(size_t)rb * NB + cb * B + cc] = s;
    }
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of the stream seeded `seed`
// is the mix of seed + (k+1) * golden-gamma.
LQ_DEV unsigned long long splitmix64(unsigned long long seed, unsigned long long k) {
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct DecideArgs {
    int crit;
    double alpha;
    int forced_k;
    unsigned long long seed;
};

// The decision of step k (one workgroup).  Special cases in order: forced
// sequence; alpha = +inf => LU; alpha = 0 => QR; zero pivot in the diagonal
// tile => QR; non-finite criterion input => QR.  Ties alpha*s == m take LU.
template <int NB>
__global__ __launch_bounds__(WG) void k_panel_decide(Ctx c, int k, DecideArgs a) {
    __shared__ double red[WG];
    __shared__ double awayj[NB];
    const int tid = threadIdx.x;
    const int mk = c.msize(k);
    const int zp = c.zpiv[k];
    // ||A_kk^{-1}||_1 over the real columns of the tile
    double inv = 0.0;
    for (int j = tid; j < mk; j += WG) {
        double s = 0.0;
        for (int rb = 0; rb < (NB < 64 ? 1 : NB / 64); ++rb) s += c.invpart[(size_t)rb * NB + j];
        inv = nmax(inv, s);
    }
    red[tid] = inv;
    for (int j = tid; j < NB; j += WG) {
        double v = 0.0;
        for (int i = k + 1; i < c.n; ++i) v = nmax(v, c.away[(size_t)i * NB + j]);
        awayj[j] = v;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int t = 1; t < WG; ++t) inv = nmax(inv, red[t]);
    double s = zp ? 0.0 : 1.0 / inv;
    double m = 0.0;
    for (int i = k + 1; i < c.n; ++i) {
        double t = c.tnorm[i];
        m = (a.crit == LUQR_CRIT_SUM) ? m + t : nmax(m, t);
    }
    int nonfinite = !(isfinite(s) && isfinite(m));
    int lu;
    double margin;
    if (a.crit == LUQR_CRIT_FORCED) {
        lu = a.forced_k != 0; margin = lu ? 1.0 : -1.0;
    } else if (isinf(a.alpha)) {
        lu = 1; margin = 1.0;
    } else if (a.alpha == 0.0) {
        lu = 0; margin = -1.0;
    } else if (zp) {
        lu = 0; margin = -1.0;
    } else if (a.crit == LUQR_CRIT_MAX || a.crit == LUQR_CRIT_SUM) {
        if (nonfinite) { lu = 0; margin = -1.0; }
        else {
            const double as = a.alpha * s;
            lu = as >= m;
            double den = fmax(fmax(as, m), 2.2250738585072014e-308);
            margin = (as - m) / den;
        }
    } else if (a.crit == LUQR_CRIT_MUMPS) {
        // estimate_max(j) starts at away_max(j) and is multiplied by the
        // growth factor of every earlier column i < j of the GEPP on the copy
        const double *W = c.W + (size_t)k * NB * NB;
        double prod = 1.0, smin = INFINITY, emax = 0.0;
        lu = 1; margin = INFINITY;
        for (int j = 0; j < mk; ++j) {
            const double pj = fabs(W[j + j * NB]);
            const double gf = pj / c.lmax[j];
            const double est = awayj[j] * prod;
            prod *= gf;
            if (!isfinite(est) || !isfinite(pj)) nonfinite = 1;
            const double ap = a.alpha * pj;
            if (!(ap >= est)) lu = 0;
            double den = fmax(fmax(ap, est), 2.2250738585072014e-308);
            margin = fmin(margin, (ap - est) / den);
            smin = fmin(smin, pj);
            emax = fmax(emax, est);
        }
        if (nonfinite) { lu = 0; margin = -1.0; }
        s = smin; m = emax;
    } else {
        const double u = (double)(splitmix64(a.seed, (unsigned long long)k) >> 11) * 0x1.0p-53;
        lu = u < a.alpha / 100.0;
        margin = a.alpha / 100.0 - u;
    }
    c.dec[k] = lu;
    c.s[k] = s;
    c.m[k] = m;
    c.margin[k] = margin;
    if (nonfinite) c.st->nonfinite = 1;
    if (lu) {
        c.st->n_lu += 1;
        if (zp && c.st->info == 0) c.st->info = (long long)k * NB + zp;
    }
}

// QR steps: Dinv_k <- R_kk^{-1} from the upper triangle of the factored tile.
template <int NB, class S>
__global__ __launch_bounds__(WG) void k_qr_rinv(Ctx c, int k) {
    if (c.dec[k] != 0) return;
    trtri_col<NB, S>((const S *)c.At + c.toff(k, k), c.Dinv + (size_t)k * NB * NB, true);
}

}  // namespace lq
