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

// Per-column exchange area, two buffers (column q uses buffer q & 1, so a
// thread may start writing column q+1 while others still read column q).
struct GetrfLds {
    double bv[2][4];
    int bi[2][4];
    int dnan[2];          // the diagonal entry of the column being eliminated is NaN
    double cand[2][4][32];// each wave's best row of the 32-column panel
    double rowA[2][32];   // the diagonal row
    int piv[32];
    int tcnt;
    int trow[64], tsrc[64];
};

// The 32 columns of a panel, one per iteration and one barrier each: before
// the barrier each wave's winner of the argmax writes its whole row (and the
// owner of the diagonal row writes that one), so after it every thread takes
// the pivot row from the winning wave's slot without a second round trip.
// The thread's rows sit in registers in rotated order: at column q, P[u][j]
// holds panel column (q + j) mod 32, so the column being eliminated is always
// P[u][0] and one small loop body serves every column; 32 rotations restore
// the original order.
template <int RPT>
LQ_DEV void lu_panel_columns(double (&P)[RPT][32], int p0, int R, GetrfLds *g, int &zp) {
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
#pragma unroll 1
    for (int q = 0; q < 32; ++q) {
        const int col = p0 + q, buf = q & 1;
        const int act = 32 - q;  // positions 0 .. act-1 hold columns q .. 31
        double v = -1.0;
        int idx = 0x7fffffff;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {  // rows ascending within the thread
            const int r = tid + 256 * u;
            if (r >= col && r < R) {
                const double a = fabs(P[u][0]);
                if (a > v) { v = a; idx = r; }
            }
            if (r == col) {
                g->dnan[buf] = P[u][0] != P[u][0];
#pragma unroll
                for (int j = 0; j < 32; ++j) g->rowA[buf][j] = P[u][j];
            }
        }
        wave_argmax(v, idx);
        if (idx != 0x7fffffff && tid == (idx & 255)) {  // this thread holds the wave's best row
#pragma unroll
            for (int u = 0; u < RPT; ++u)
                if ((idx >> 8) == u) {
#pragma unroll
                    for (int j = 0; j < 32; ++j) g->cand[buf][w][j] = P[u][j];
                }
        }
        if (l == 0) { g->bv[buf][w] = v; g->bi[buf][w] = idx; }
        __syncthreads();
        double wv[4];
        int wi[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) { wv[t] = g->bv[buf][t]; wi[t] = g->bi[buf][t]; }
        const bool dnan = g->dnan[buf] != 0;
        v = wv[0];
        idx = wi[0];
        int win = 0;
#pragma unroll
        for (int t = 1; t < 4; ++t) {
            const bool take = (wv[t] > v) | ((wv[t] == v) & (wi[t] < idx));
            v = take ? wv[t] : v;
            idx = take ? wi[t] : idx;
            win = take ? t : win;
        }
        // The scan that defines the pivot starts at the diagonal and moves to
        // a later row only if its magnitude is strictly larger, so a NaN on
        // the diagonal stays the pivot (and NaNs below it are never chosen); a
        // column of exact zeros on and below the diagonal is skipped.
        const bool zero = !dnan && !(v > 0.0);
        const int piv = (zero || dnan) ? col : idx;
        if (tid == 0) g->piv[q] = piv;
        zp = (zero && zp == 0) ? col + 1 : zp;  // the same in every thread
        if (!zero) {
            const double *rowA = g->rowA[buf];
            const double *rowB = piv == col ? rowA : g->cand[buf][win];
            const double pv = rowB[0];
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int r = tid + 256 * u;
                if (r == col || r == piv) {  // the interchange
                    const double *sr = r == col ? rowB : rowA;
#pragma unroll
                    for (int j = 0; j < 32; ++j) P[u][j] = sr[j];
                }
                if (r > col && r < R) {
                    const double lr = P[u][0] / pv;
                    P[u][0] = lr;
                    // positions act.. hold earlier columns' multipliers: their
                    // factor is zero (lr is finite whenever the step is kept:
                    // a NaN pivot sends the step to QR, which discards W)
#pragma unroll
                    for (int j = 1; j < 32; ++j) {
                        const long long mk = j < act ? -1ll : 0ll;  // bit mask: no branch per position
                        P[u][j] -= lr * __longlong_as_double(__double_as_longlong(rowB[j]) & mk);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const double t0 = P[u][0];
#pragma unroll
            for (int j = 0; j < 31; ++j) P[u][j] = P[u][j + 1];
            P[u][31] = t0;
        }
    }
}

// The row moves of one panel's 32 interchanges (row p0 + q with piv[q], in
// order), built by one wave with a lane per touched row: lanes 0..31 stand
// for rows p0..p0+31, lane 32 + q for piv[q] when it lies below the panel and
// first appears at q.  Each lane carries the position (before the panel) of
// the row now at its own position; the interchanges pass these between lanes
// in registers.  Result: trow[t] receives row tsrc[t], and the running
// permutation gsrc (position -> original row) is composed with the moves.
LQ_DEV void panel_moves(int p0, GetrfLds &g, int *gsrc) {
    const int l = lane_id();
    int pv[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) pv[q] = g.piv[q];  // the same in every lane
    const int b = g.piv[l & 31];
    int first = 32;
#pragma unroll
    for (int q = 31; q >= 0; --q) first = pv[q] == b ? q : first;
    const bool valid = l < 32 || (b >= p0 + 32 && first == l - 32);
    const int key = l < 32 ? p0 + l : b;
    int cont = key;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int a = p0 + q, bq = __builtin_amdgcn_readfirstlane(pv[q]);
        if (bq != a) {
            const int lb = bq < p0 + 32 ? bq - p0 : 32 + __builtin_amdgcn_readlane(first, 32 + q);
            const int ca = __builtin_amdgcn_readlane(cont, q), cb = __builtin_amdgcn_readlane(cont, lb);
            cont = l == q ? cb : (l == lb ? ca : cont);
        }
    }
    const bool mv = valid && cont != key;
    const unsigned long long bal = __ballot(mv);
    const int pos = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
    const int gs = mv ? gsrc[cont] : 0;  // every lane reads before any writes
    if (mv) {
        g.trow[pos] = key;
        g.tsrc[pos] = cont;
        gsrc[key] = gs;
    }
    if (l == 0) g.tcnt = __popcll(bal);
}

// The same elimination runs on the diagonal tile alone (R = NB rows, W the
// step's copy, ld NB) or on the stacked diagonal domain (R = d NB rows of the
// tiles k, k+p, ..., W = c.WD, ld DR): the pivot of each column is searched
// over all R rows.  RPT = rows per thread / 256 >= R / 256.
// The tile variant (RPT = 1, n_b <= 256) stages L21 whole and U12 in chunks
// of UC columns for its MFMA update, with L11 in the U12 area (it is done with
// before U12 is staged): about 80 KB at n_b = 256, so the workgroup fits on a
// compute unit beside a trailing-update workgroup of the previous step.
template <int NB, int RPT> struct GetrfSmem {
    static constexpr bool MF = NB <= 256 && RPT == 1;  // A22 on FP64 MFMA
    static constexpr int LDL = NB - 31;                 // L21 rows (at most NB - 32), odd stride
    static constexpr int UC = 64;                       // U12 columns per staged chunk
    static constexpr int UBN = UC * 33 > 32 * 33 ? UC * 33 : 32 * 33;
    static constexpr int BUFN = MF ? 32 * LDL + UBN : 32 * 33;
    double buf[BUFN];  // L21 / U12 staging of the trailing update
    double L11x[MF ? 1 : 32 * 33];
    LQ_DEV double *L11() { if constexpr (MF) return buf + 32 * LDL; else return L11x; }
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
    double *buf = sm.buf, *L11 = sm.L11();
    int *src = sm.src;
    unsigned long long *lmx = sm.lmx;
    GetrfLds &g = sm.g;
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    double *W = dom ? c.WD : c.W + (size_t)k * NB * NB;
    const S *A = (const S *)c.At + c.toff(k, k);
    for (int e = tid; e < NB; e += WG) lmx[e] = 0ull;
    for (int r = tid; r < R; r += WG) src[r] = r;  // running permutation of the rows
    int zp = 0;                                     // first zero pivot column + 1
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
    // copy A_kk -> W (FP64) and its column maxima (MUMPS local_max): four
    // consecutive entries of one column per load, 16 loads in flight
    struct alignas(4 * sizeof(S)) S4 { S v[4]; };
    constexpr int NV = NB * NB / 4;
    for (int v0 = 0; v0 < NV; v0 += 16 * WG) {
        S4 a[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int vi = v0 + t * WG + tid;
            if (vi < NV) a[t] = ((const S4 *)A)[vi];
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int vi = v0 + t * WG + tid;
            double m = 0.0;
            if (vi < NV) {
                d2 x0, x1;
                x0[0] = (double)a[t].v[0]; x0[1] = (double)a[t].v[1];
                x1[0] = (double)a[t].v[2]; x1[1] = (double)a[t].v[3];
                ((d2 *)W)[2 * vi] = x0;
                ((d2 *)W)[2 * vi + 1] = x1;
                m = nmax(nmax(fabs(x0[0]), fabs(x0[1])), nmax(fabs(x1[0]), fabs(x1[1])));
            }
            // non-negative doubles (and NaN above them) order as their bit patterns
            if constexpr (NB >= 256) {
                m = wave_nmax(m);  // a wave covers 256 consecutive rows of one column
                if (l == 0 && vi < NV) atomicMax(&lmx[4 * vi / NB], (unsigned long long)__double_as_longlong(m));
            } else if (vi < NV) {
                atomicMax(&lmx[4 * vi / NB], (unsigned long long)__double_as_longlong(m));
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
        lu_panel_columns<RPT>(P, p0, R, &g, zp);
        __syncthreads();  // the last column's pivot is recorded
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
            if constexpr (GetrfSmem<NB, RPT>::MF) {  // L21 for the MFMA update, row r at r - (p0 + 32)
                if (r >= p0 + 32 && r < NB) {
#pragma unroll
                    for (int j = 0; j < 32; ++j) buf[j * GetrfSmem<NB, RPT>::LDL + r - p0 - 32] = P[u][j];
                }
            }
        }
        if (tid < 32) c.ipiv[(size_t)k * NB + p0 + tid] = g.piv[tid];
        if (w == 0) panel_moves(p0, g, src);  // rows moved by the panel's interchanges
        __syncthreads();
        {   // the panel's interchanges on the columns outside it: a wave per
            // column (its moved rows lie in one column), a lane per moved row;
            // wave w takes columns w, w + 4, ..., GB of them loaded before any
            // is written
            constexpr int NC = NB / 4, GB = NC < 32 ? NC : 32;
            const int cnt = g.tcnt;
            const int ts = l < cnt ? g.tsrc[l] : 0, tr = l < cnt ? g.trow[l] : 0;
#pragma unroll 1
            for (int b0 = 0; b0 < NC; b0 += GB) {
                double v[GB];
#pragma unroll
                for (int b = 0; b < GB; ++b) {
                    const int cc = 4 * (b0 + b) + w;
                    const bool mv = l < cnt && !(cc >= p0 && cc < p0 + 32);
                    v[b] = mv ? W[ts + (size_t)cc * ldw] : 0.0;
                }
#pragma unroll
                for (int b = 0; b < GB; ++b) {
                    const int cc = 4 * (b0 + b) + w;
                    const bool mv = l < cnt && !(cc >= p0 && cc < p0 + 32);
                    if (mv) W[tr + (size_t)cc * ldw] = v[b];
                }
            }
        }
        __syncthreads();
        if (p0 + 32 < NB) {
            for (int cc = p0 + 32 + tid; cc < NB; cc += WG) {  // U12 = L11^{-1} A12
                double x[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) x[q] = W[p0 + q + (size_t)cc * ldw];
#pragma unroll
                for (int q = 0; q < 32; ++q) {
#pragma unroll
                    for (int r = q + 1; r < 32; ++r) x[r] -= L11[q * 33 + r] * x[q];
                    // keep the scheduler from hoisting every L11 load (register pressure)
                    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int q = 0; q < 32; ++q) W[p0 + q + (size_t)cc * ldw] = x[q];
            }
            __syncthreads();
            if constexpr (GetrfSmem<NB, RPT>::MF) {
                // A22 -= L21 U12 on FP64 MFMA: L21 (rows p0+32.., 32 cols, staged in LDS
                // with the panel's write-back), U12 in chunks of UC columns
                constexpr int LDL = GetrfSmem<NB, RPT>::LDL, UC = GetrfSmem<NB, RPT>::UC;
                double *Ls = buf;                 // [32][LDL], row r at r - r0
                double *Ub = buf + 32 * LDL;      // [UC][33]
                const int r0 = p0 + 32, m = NB - r0;
                const int nbk = m / 16;
                const int gq = l >> 4, i16 = l & 15;
                for (int c0 = r0; c0 < NB; c0 += UC) {
                    const int nc = NB - c0 < UC ? NB - c0 : UC;
                    for (int e = tid; e < 32 * nc; e += WG) Ub[(e / 32) * 33 + e % 32] = W[p0 + e % 32 + (c0 + e / 32) * NB];
                    __syncthreads();
                    // a wave takes 16-row blocks w, w + 4, ... across the chunk's
                    // columns; the chunk's B operands stay in registers for all of them
                    const int ncb = nc / 16;
                    double bop[UC / 16][8];
#pragma unroll
                    for (int cb = 0; cb < UC / 16; ++cb)
#pragma unroll
                        for (int ks = 0; ks < 8; ++ks)
                            bop[cb][ks] = cb < ncb ? Ub[(16 * cb + i16) * 33 + 4 * ks + gq] : 0.0;
                    // the next row block's C tiles are loaded while this one's are computed
                    d4 cur[UC / 16], nxt[UC / 16];
                    auto load_c = [&](int rb, d4 (&cv)[UC / 16]) {
#pragma unroll
                        for (int cb = 0; cb < UC / 16; ++cb)
                            if (cb < ncb && rb < nbk) {
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    cv[cb][r] = W[(r0 + 16 * rb + Tr<P64>::drow(gq, r)) + (c0 + 16 * cb + i16) * NB];
                            }
                    };
                    load_c(w, cur);
                    for (int rb = w; rb < nbk; rb += 4) {
                        const int br = r0 + 16 * rb;
                        load_c(rb + 4, nxt);
                        double aop[8];
#pragma unroll
                        for (int ks = 0; ks < 8; ++ks) aop[ks] = -Ls[(4 * ks + gq) * LDL + br - r0 + i16];
#pragma unroll
                        for (int cb = 0; cb < UC / 16; ++cb)
                            if (cb < ncb) {
#pragma unroll
                                for (int ks = 0; ks < 8; ++ks) cur[cb] = Tr<P64>::mma(aop[ks], bop[cb][ks], cur[cb]);
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    W[(br + Tr<P64>::drow(gq, r)) + (c0 + 16 * cb + i16) * NB] = cur[cb][r];
                            }
#pragma unroll
                        for (int cb = 0; cb < UC / 16; ++cb) cur[cb] = nxt[cb];
                    }
                    __syncthreads();
                }
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
    // permutation of the whole tile (or stacked domain): (P A)(r,:) = A(src[r],:),
    // composed panel by panel above
    if (tid == 0) c.zpiv[k] = zp;
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

// Column sums and column maxima of |A_ik| (one workgroup per tile).  A wave
// takes columns w, w + 4, ...; CPW of them are loaded before any is reduced,
// so that enough loads are in flight to cover the memory latency.
// cs: NB doubles of LDS (the caller's: this runs inside launches whose other
// workgroups need all of theirs).
template <int NB, class S>
LQ_DEV void tile_norms(const Ctx &c, int k, int i, double *cs) {
    const int l = lane_id(), w = wave_id();
    const S *A = (const S *)c.At + c.toff(i, k);
    constexpr int RPL = NB >= 64 ? NB / 64 : 1;  // rows per lane
    constexpr int CPW = NB >= 256 ? 8 : 16;      // columns per wave in flight
    for (int c0 = w; c0 < NB; c0 += 4 * CPW) {
        double a[CPW][RPL];
#pragma unroll
        for (int t = 0; t < CPW; ++t)
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
                const int col = c0 + 4 * t, r = l + 64 * u;
                a[t][u] = (col < NB && r < NB) ? fabs((double)A[r + col * NB]) : 0.0;
            }
#pragma unroll
        for (int t = 0; t < CPW; ++t) {
            double sum = 0.0, mx = 0.0;
#pragma unroll
            for (int u = 0; u < RPL; ++u) { sum += a[t][u]; mx = nmax(mx, a[t][u]); }
            sum = wave_sum(sum);
            mx = wave_nmax(mx);
            const int col = c0 + 4 * t;
            if (l == 0 && col < NB) { cs[col] = sum; c.away[(size_t)i * NB + col] = mx; }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int col = 0; col < NB; ++col) t = nmax(t, cs[col]);
        c.tnorm[i] = t;
    }
}

// GEPP of the diagonal tile (RPT = 1) or of the stacked diagonal domain and
// of 512-row tiles (RPT = 2) in workgroup 0; the tile norms of the criterion
// (workgroups 1.., tile k + blockIdx.x; the tiles of a diagonal domain are
// measured after its elimination), which do not depend on it, run beside
// it in the same launch, so they cost nothing on the step's critical path.
// The tile variant is held to half a SIMD's registers, so that it fits on a
// compute unit beside a trailing-update workgroup of the previous step.
// early = 1: after a QR step k-1 the tile's GEPP ran inside that step (its
// last workgroup) and the tile norms run beside the triangular inverses
// (k_panel_trtri), so the launch has nothing to do.
template <int NB, class S, int RPT>
__global__ __launch_bounds__(WG, RPT == 1 ? 2 : 1) void k_panel_getrf(Ctx c, int k, int early) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(GetrfSmem<NB, RPT>)];
    if (early && c.dec[k - 1] == 0) return;
    if (blockIdx.x > 0) {
        const int i = k + (int)blockIdx.x;
        if (!c.indom(k, i)) tile_norms<NB, S>(c, k, i, (double *)smem);
        return;
    }
    getrf_core<NB, S, RPT>(c, k, smem);
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

// Panel: NB/2 workgroups; the first NB/4 invert U (into Dinv_k), the next
// NB/4 invert L (into Linv_k), both from the GETRF copy W_k.  early = 1: the
// launch has n-k-1 more workgroups, which compute the tile norms of the
// criterion when step k-1 was a QR step (k_panel_getrf's otherwise).
template <int NB, class S>
__global__ __launch_bounds__(WG) void k_panel_trtri(Ctx c, int k, int early) {
    if ((int)blockIdx.x >= NB / 2) {
        __shared__ double cs[NB];
        if (early && c.dec[k - 1] == 0) tile_norms<NB, S>(c, k, k + 1 + (int)blockIdx.x - NB / 2, cs);
        return;
    }
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
    if (a.crit == LUQR_CRIT_MUMPS)
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

// ---------------------------------------------------------------------------
// Panel of variant A2 (Sec. 2.3).  Its Factor is a QR factorization of A_kk;
// here it runs in FP64 on a working copy W_k (k_a2_copy, k_a2_geqrt), so the
// criterion's ||A_kk^{-1}||_1 is taken from FP64 factors in every storage
// precision, as A1's is from its FP64 GEPP.  The copy is no backup: nothing is
// restored from it, and the storage tile receives the rounded V\R and T
// (k_a2_commit) for the branch that follows, LU or QR alike.
// ---------------------------------------------------------------------------
template <int NB, class S>
__global__ __launch_bounds__(WG) void k_a2_copy(Ctx c, int k) {
    const S *A = (const S *)c.At + c.toff(k, k);
    double *W = c.W + (size_t)k * NB * NB;
    for (int e = blockIdx.x * WG + threadIdx.x; e < NB * NB; e += gridDim.x * WG) W[e] = (double)A[e];
}

// Last of the A2 panel (both branches use it): Dinv_k <- R^{-1} from the FP64
// R of the GEQRT on W_k (overwriting the T factor kept there).
template <int NB>
__global__ __launch_bounds__(WG) void k_a2_rinv(Ctx c, int k) {
    trtri_col<NB, double>(c.W + (size_t)k * NB * NB, c.Dinv + (size_t)k * NB * NB, true);
}

// After k_a2_qt (which reads T from the Dinv_k slot): tile (k,k) <- V\R and
// the diagonal IB-blocks of its T factor <- T, both rounded to storage.
template <int NB, class S>
__global__ __launch_bounds__(WG) void k_a2_commit(Ctx c, int k) {
    S *A = (S *)c.At + c.toff(k, k);
    S *T = (S *)c.Tf + c.tqoff(k, k);
    const double *W = c.W + (size_t)k * NB * NB;
    const double *T64 = c.Dinv + (size_t)k * NB * NB;
    for (int e = blockIdx.x * WG + threadIdx.x; e < NB * NB; e += gridDim.x * WG) {
        A[e] = (S)W[e];
        const int r = e % NB, col = e / NB;
        if (r / IB == col / IB) T[e] = (S)T64[e];
    }
}

// Linv_k <- Q_kk^T in FP64, so that the criterion's ||A_kk^{-1}||_1 =
// ||R^{-1} Q^T||_1, the Apply (A_kj <- Q^T A_kj) and the solve's z_k = Q^T y_k
// are the A1 products with L^{-1}; perm_k and ipiv_k <- identity; zpiv_k <-
// first zero on R's diagonal (1-based) over the tile's real columns.  Q = Q_0
// Q_1 .. Q_{B-1} with Q_b = I - V_b T_b V_b^T the IB-column blocks of the
// GEQRT (V unit lower in W_k, T_b the diagonal blocks of its T factor, in the
// Dinv_k slot), so Q^T is the identity with Q_0^T, Q_1^T, .. applied in turn.
// Grid NB/16: each workgroup forms 16 columns, held in LDS with the current
// block of V.
template <int NB>
__global__ __launch_bounds__(WG) void k_a2_qt(Ctx c, int k) {
    static_assert(IB == 16, "one thread per (reflector, column) of a block");
    __shared__ double C[NB * 16];   // C[r*16 + col]: column cb*16 + col of the running product
    __shared__ double Vs[IB * NB];  // Vs[q*NB + r] = V(r, c0 + q), zeros and ones explicit
    __shared__ double Ts[IB * IB], Wb[IB * 16], Wt[IB * 16];
    const int tid = threadIdx.x, cb = blockIdx.x;
    const double *A = c.W + (size_t)k * NB * NB;
    const double *T = c.Dinv + (size_t)k * NB * NB;
    for (int e = tid; e < NB * 16; e += WG) C[e] = (e / 16 == cb * 16 + e % 16) ? 1.0 : 0.0;
    const int p = tid / 16, col = tid % 16;
    for (int b = 0; b < NB / IB; ++b) {
        const int c0 = b * IB;
        for (int e = tid; e < IB * NB; e += WG) {
            const int q = e / NB, r = e % NB;
            Vs[e] = r < c0 + q ? 0.0 : (r == c0 + q ? 1.0 : A[r + (size_t)(c0 + q) * NB]);
        }
        Ts[tid] = T[(c0 + tid % IB) + (size_t)(c0 + tid / IB) * NB];  // Ts[q*IB + p] = T(p, q)
        __syncthreads();
        // W = V_b^T C over rows c0.. (V's zeros above its diagonal included),
        // in four interleaved partial sums
        double w4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = c0; r < NB; r += 4)
#pragma unroll
            for (int u = 0; u < 4; ++u) w4[u] += Vs[p * NB + r + u] * C[(r + u) * 16 + col];
        Wb[p * 16 + col] = (w4[0] + w4[1]) + (w4[2] + w4[3]);
        __syncthreads();
        double wt = 0.0;  // T_b^T W: (T^T)(p, q) = T(q, p), nonzero for q <= p
        for (int q = 0; q <= p; ++q) wt += Ts[p * IB + q] * Wb[q * 16 + col];
        Wt[p * 16 + col] = wt;
        __syncthreads();
        // C -= V_b (T_b^T W); every row this thread updates is in column col
        // (WG is a multiple of 16), so that column of T_b^T W stays in registers
        double wc[IB];
#pragma unroll
        for (int q = 0; q < IB; ++q) wc[q] = Wt[q * 16 + col];
        static_assert(IB * 16 % WG == 0, "row c0 starts a whole pass of the workgroup");
        for (int e = tid + c0 * 16; e < NB * 16; e += WG) {  // rows c0..; above them V_b is zero
            const int r = e / 16;
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < IB; ++q) acc += Vs[q * NB + r] * wc[q];
            C[e] -= acc;
        }
        __syncthreads();
    }
    double *Q = c.Linv + (size_t)k * NB * NB;
    for (int e = tid; e < NB * 16; e += WG) Q[e % NB + (size_t)(cb * 16 + e / NB) * NB] = C[(e % NB) * 16 + e / NB];
    if (cb == 0) {
        for (int r = tid; r < NB; r += WG) c.perm[(size_t)k * NB + r] = c.ipiv[(size_t)k * NB + r] = r;
        if (tid == 0) {
            int zp = 0;
            const int mk = c.msize(k);
            for (int j = 0; j < mk && !zp; ++j)
                if (A[j + (size_t)j * NB] == 0.0) zp = j + 1;
            c.zpiv[k] = zp;
        }
    }
}

}  // namespace lq
