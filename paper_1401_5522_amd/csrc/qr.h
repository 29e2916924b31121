// QR step with TS kernels and a flat reduction tree (Alg. 3 and 4a: the
// eliminator of every A_ik is A_kk), run only when the device-side decision
// of step k says QR.  One launch per step:
//   workgroups 0..nb/IB-1 (producers): workgroup b factors column block b
//     (IB columns) of GEQRT(A_kk) and then of TSQRT(R_kk, A_ik) for
//     i = k+1..n-1, owning row block b of R_kk throughout.  Unit (i, b) needs
//     the trailing update of unit (i, b-1) (flag) and R's row block b (its own
//     previous unit), so the chain advances as a wavefront over (i, b);
//     flag[i][b] = k+1 publishes the block reflector Y_ib, T_ib;
//   the other workgroups (consumers): one 64-column strip of one trailing
//     tile column j; UNMQR on the strip of A_kj, then TSMQR(i) on the strips of
//     (A_kj, A_ij), block reflector by block reflector as each is published.
// A consumer keeps the strip of A_ij in MFMA accumulator registers (each wave
// owns 16 columns over all nb rows) and the strip of A_kj in LDS (or, where
// LDS is short, in place in global memory) for the whole chain, so A_kj never
// leaves the chip between the n-k-1 updates it receives.
// The panel work of one unit grows with IB^2 (IB columns, each reducing over
// IB columns) while the chain gains one unit per block, so IB = 16 keeps the
// producer wavefront short.
// Reflectors use the LAPACK convention: beta = -sign(alpha)||x||, tau = 0
// when the tail is zero.  The QR step builds the compact-WY factor per IB
// columns: block b of T(i,k) is the diagonal block (b*IB.., b*IB..) of the
// nb x nb factor of tile (i,k); k_qr_gram and k_qr_tfull fill the blocks above
// the diagonal afterwards, so the solve can apply each tile's reflectors as
// one block (I - V T V^T).
#pragma once
#include <utility>

#include "mma.h"

namespace lq {

template <class S> LQ_DEV S sq(S x) { return x * x; }

// x = hi + lo to about 2^-16 relative, hi and lo rounded to BF16.
LQ_DEV __bf16 bf_hi(float x) { return (__bf16)x; }
LQ_DEV __bf16 bf_lo(float x) { return (__bf16)(x - (float)(__bf16)x); }

template <int NB> constexpr int qr_rpt() { return NB > 256 ? 2 : 1; }  // panel rows per thread

// ---------------------------------------------------------------------------
// Producer panel: Householder QR of one IB-column block (c0 = b*IB) with the
// panel held in registers, thread t owning tile rows t and t+256.
//   TS = false: GEQRT panel of the tile A (rows c0.., unit-lower V in place).
//   TS = true:  TSQRT panel of [R; A]: R's diagonal block (Rb, LDS, row-major) holds the
//               pivots, A's whole column is the reflector tail Y.
// Column q runs as its own instantiation (compile-time q), so every register
// index is static.  One cross-workgroup reduction per column: with x the
// unscaled tail of column q (after reflectors 0..q-1), it sums x^T x, x^T a_j
// for the columns j > q still to update, and x^T v_j for the reflectors
// j < q.  The Householder scale s = 1/(alpha - beta) is applied afterwards:
// v_q^T a_j = base_j + s x^T a_j, where base_j is the pivot-row entry (R(q, j)
// for TS, A(pivot, j) for GEQRT), and the same form gives the Gram entries
// v_j^T v_q that extend the compact-WY factor T.  The reduction of column q+1
// is formed right after column q's update (partial sums ping-pong between two
// LDS buffers); one wave turns the sums into the reflector, so each column
// costs two barriers.
// On return Ys holds V (explicit zeros/ones for GEQRT) and Ts holds T.
// ---------------------------------------------------------------------------
// A block reflector V (nb x IB) staged in LDS is kept twice: column-major
// (Yc[q*LDY + r], the operand of W = V^T C) and row-major (Yr[r*LDQ + q], the
// operand of C -= V W).  With LDY = nb+4 and LDQ = IB+4 the sixteen lanes of
// each quarter-wave read sixteen disjoint 16-byte bank groups, so both MFMA
// operands load as conflict-free 128-bit reads.  vblk = both copies.
template <int NB> constexpr int qr_ldy() { return NB + 4; }
constexpr int LDQ = IB + 4;
template <int NB> constexpr int qr_vblk() { return IB * qr_ldy<NB>() + NB * LDQ; }
template <int NB, class S> LQ_DEV S *vrow(S *Ys) { return Ys + IB * qr_ldy<NB>(); }
template <int NB, class S> LQ_DEV const S *vrow(const S *Ys) { return Ys + IB * qr_ldy<NB>(); }
template <int NB, class S> LQ_DEV void put_v(S *Ys, int r, int q, S v) {
    Ys[q * qr_ldy<NB>() + r] = v;
    vrow<NB>(Ys)[r * LDQ + q] = v;
}

struct PanelLds {
    double red[2][IB * 4];  // [buffer][j][wave]: the waves' partial sums (values of type S)
    double prow[2][IB];     // GEQRT: pivot row of the column being reduced (type S)
    double pmax[4];         // per-wave largest magnitude of the panel block
    double dcol[IB];        // column q: d_j = v_q^T a_j (j > q), v_j^T v_q (j < q) (type S)
    double wcol[IB];        // column q: w_j = tau d_j, the rank-1 update's row (type S)
    double sc[4];           // column q: scal, tau, beta (type S)
};

template <class S> LQ_DEV S rlane(S v, int lane) {
    if constexpr (sizeof(S) == 4) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    else
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                                __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Partial sums of column q's reduction into pl->red[q & 1]; for GEQRT the
// owner of the pivot row also publishes it.
template <int NB, class S, bool TS, int Q>
LQ_DEV void qr_reduce(S (&P)[qr_rpt<NB>()][IB], int c0, PanelLds *pl) {
    constexpr int RPT = qr_rpt<NB>();
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    const int pr = c0 + Q;
    S x[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = tid + 256 * u;
        x[u] = (TS ? r < NB : (r > pr && r < NB)) ? P[u][Q] : (S)0;
        if (!TS && r == pr) {
#pragma unroll
            for (int j = 0; j < IB; ++j) ((S *)pl->prow[Q & 1])[j] = P[u][j];
        }
    }
#pragma unroll
    for (int half = 0; half < IB / 16; ++half) {
        S part[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * half + jj;
            S acc = 0;
#pragma unroll
            for (int u = 0; u < RPT; ++u) acc += x[u] * P[u][j];
            part[jj] = acc;
        }
        const S tot = xreduce16<S>(part);
        if ((l & 3) == 0) ((S *)pl->red[Q & 1])[(16 * half + (l >> 2)) * 4 + w] = tot;
    }
}

// Column q of the panel, between two barriers.  Wave 0 turns the reduced sums
// into the reflector: lane j (j < IB) forms f_j = x^T a_j from the four waves'
// partials and the pivot-row entry base_j (row q of R's row-major block for
// TS), every lane takes f_q and base_q from lane q for the norm, and lane j
// forms d_j and w_j = tau d_j and, for TS, writes R(q, j) at once (no other
// wave reads R's row q).  A barrier then hands scal, tau, beta, d and w to
// every thread for the rank-1 update of its rows and the new column of T.
// The products and lane sums are in the storage precision on a panel block
// scaled to a largest magnitude near 1 (panel_qr), so they neither overflow
// nor underflow; a column whose remaining norm is below 2^-50 (FP32) or
// 2^-500 (FP64) of that is left as it is (tau = 0), as for an exactly zero
// one.
template <int NB, class S, bool TS, int Q>
LQ_DEV void qr_column(S (&P)[qr_rpt<NB>()][IB], int c0, S *Rb, S *Ts, PanelLds *pl) {
    constexpr int RPT = qr_rpt<NB>();
    constexpr S TINY = sizeof(S) == 4 ? (S)0x1.0p-100 : (S)0x1.0p-1000;  // of the squared norm
    const int tid = threadIdx.x, l = lane_id();
    const int pr = c0 + Q;  // GEQRT pivot row
    S *dcol = (S *)pl->dcol, *wcol = (S *)pl->wcol, *sc = (S *)pl->sc;
    if (tid < 64) {
        const int j = l & (IB - 1);
        const S *red = (const S *)pl->red[Q & 1];
        const S fj = (red[j * 4] + red[j * 4 + 1]) + (red[j * 4 + 2] + red[j * 4 + 3]);
        const S bj = TS ? (j >= Q ? Rb[Q * IB + j] : (S)0) : ((const S *)pl->prow[Q & 1])[j];
        const S ss = rlane(fj, Q), alpha = rlane(bj, Q);
        S tau = 0, beta = alpha, scal = 1;
        if (ss >= TINY) {
            const S nrm = sqrt(alpha * alpha + ss);
            beta = alpha >= (S)0 ? -nrm : nrm;
            const S g = alpha - beta;  // |g| >= nrm
            scal = (S)1 / g;
            tau = -g / beta;
        }
        const S dj = j == Q ? (S)0 : bj + scal * fj;
        const S wj = j > Q ? tau * dj : (S)0;
        if (l < IB) {
            dcol[j] = dj;
            wcol[j] = wj;
            if (TS && j >= Q) Rb[Q * IB + j] = j == Q ? beta : bj - wj;
        }
        if (l == 0) { sc[0] = scal; sc[1] = tau; sc[2] = beta; }
    }
    __syncthreads();
    const S scal = sc[0], tau = sc[1];
    S vq[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = tid + 256 * u;
        const bool tail = TS ? r < NB : (r > pr && r < NB);
        vq[u] = tail ? P[u][Q] * scal : ((!TS && r == pr) ? (S)1 : (S)0);
        if (tail) P[u][Q] = vq[u];
        if (!TS && r == pr) P[u][Q] = sc[2];
    }
    if (tau != (S)0) {
#pragma unroll
        for (int j = Q + 1; j < IB; ++j) {
            const S wj = wcol[j];
#pragma unroll
            for (int u = 0; u < RPT; ++u) P[u][j] -= vq[u] * wj;
        }
    }
    // T(0:q, q) = -tau T(0:q, 0:q) G(0:q, q), with G(p, q) = v_p^T v_q = d_p;
    // the strictly lower part of T is stored as zeros
    if (tid < Q) {
        S acc = 0;
#pragma unroll
        for (int p = 0; p < Q; ++p) acc += Ts[p * IB + tid] * dcol[p];
        Ts[Q * IB + tid] = -tau * acc;
    } else if (tid < IB) {
        Ts[Q * IB + tid] = tid == Q ? tau : (S)0;
    }
    if constexpr (Q + 1 < IB) {
        qr_reduce<NB, S, TS, Q + 1>(P, c0, pl);
        __syncthreads();  // column q+1's sums and pivot row, R's row q+1, T's column q are visible
    }
}

template <int NB, class S, bool TS, int... Qs>
LQ_DEV void qr_columns(S (&P)[qr_rpt<NB>()][IB], int c0, S *Rb, S *Ts, PanelLds *pl,
                       std::integer_sequence<int, Qs...>) {
    qr_reduce<NB, S, TS, 0>(P, c0, pl);
    __syncthreads();
    (qr_column<NB, S, TS, Qs>(P, c0, Rb, Ts, pl), ...);
}

// Power-of-two scaling: the block (and, for TS, R's diagonal block) is
// multiplied by 2^-e, e the exponent of its largest magnitude, before the
// columns are reduced, and the R entries it produces are multiplied back by
// 2^e.  Multiplying by a power of two is exact, and the reflectors V, T and
// tau do not depend on the scale, so the result equals the unscaled
// computation wherever that one neither overflows nor underflows; products
// of entries of a block near 1 in magnitude cannot overflow, and only
// entries 2^-60 below the block's largest one can underflow, which is far
// below the storage rounding of the block (Householder QR is normwise
// backward stable).
// TT (with TS): the bottom tile is upper triangular (TTQRT of Alg. 4b): only
// its entries on and above the diagonal are read and written, the rest are
// zeros of the computation (the tile keeps other data there), and the
// reflector tails come out upper triangular.
template <int NB, class S, bool TS, bool TT = false>
LQ_DEV void panel_qr(S *A, int c0, S *Rb, S *Ys, S *Ts, PanelLds *pl) {
    static_assert(TS || !TT, "a TT panel is a TS panel on a triangular tile");
    constexpr int RPT = qr_rpt<NB>();
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    S P[RPT][IB];
    double mx = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = tid + 256 * u;
#pragma unroll
        for (int q = 0; q < IB; ++q) {
            P[u][q] = (r < NB && (TS || r >= c0) && (!TT || r <= c0 + q)) ? A[r + (c0 + q) * NB] : (S)0;
            mx = fmax(mx, fabs((double)P[u][q]));
        }
    }
    static_assert(IB * IB == WG, "R's diagonal block has one entry per thread");
    if (TS) mx = fmax(mx, fabs((double)Rb[tid]));
    mx = wave_max(mx);
    if (l == 0) pl->pmax[w] = mx;
    __syncthreads();
    mx = fmax(fmax(pl->pmax[0], pl->pmax[1]), fmax(pl->pmax[2], pl->pmax[3]));
    const int e = (mx > 0.0 && mx <= 1.7976931348623157e308) ? ilogb(mx) : 0;
    const int ec = e < -120 ? -120 : (e > 120 ? 120 : e);
    const S down = (S)ldexp(1.0, -ec), up = (S)ldexp(1.0, ec);
#pragma unroll
    for (int u = 0; u < RPT; ++u)
#pragma unroll
        for (int q = 0; q < IB; ++q) P[u][q] *= down;
    if (TS) Rb[tid] *= down;  // read by other threads only after the first barrier of qr_columns
    qr_columns<NB, S, TS>(P, c0, Rb, Ts, pl, std::make_integer_sequence<int, IB>{});
    if (TS) {
        __syncthreads();  // every column's writes of R are in place
        Rb[tid] *= up;
    } else {
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int r = tid + 256 * u;
#pragma unroll
            for (int q = 0; q < IB; ++q)
                if (r >= c0 && r <= c0 + q) P[u][q] *= up;  // R's rows of this block (beta on the diagonal)
        }
    }
    // write the panel back and expose V to the trailing update
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int r = tid + 256 * u;
        if (r >= NB) continue;
#pragma unroll
        for (int q = 0; q < IB; ++q) {
            if ((TS || r >= c0) && (!TT || r <= c0 + q)) A[r + (c0 + q) * NB] = P[u][q];
            S v;
            if (TS) v = P[u][q];
            else v = r < c0 + q ? (S)0 : (r == c0 + q ? (S)1 : P[u][q]);
            put_v<NB>(Ys, r, q, v);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Consumer: apply one block reflector (I - V T V^T)^T to a wave's 16-column
// slice.  `bot` holds all nb rows of the slice of the tile being eliminated
// into, in MFMA accumulator layout; when HAS_TOP, `top` points at the
// eliminator row tile's column for this lane (element of row r at top[r])
// and only its rows [c0, c0+IB) take part (TS structure: V = [E; Y]); they
// are read and written in place.  Without HAS_TOP the reflector lives
// entirely in `bot`'s rows (UNMQR; V given explicitly).
// Ys holds both LDS copies of V (put_v), Ts[q*IB + p] = T(p, q).
// W = V^T bot accumulates in two independent chains (even and odd row
// blocks); the top rows are added afterwards, so their load is off the chain.
// PRE: every V operand of both phases is read before the first MFMA (the
// batched kernel's 32/64 tiles).  Otherwise (k_qr_step: at nb >= 256 the bulk
// loads would exceed the registers) each 128-bit operand is read just before
// its MFMAs, and a second workgroup on the CU covers the latency.
// ---------------------------------------------------------------------------
template <int NB, int P, bool HAS_TOP, bool PRE = true>
LQ_DEV void apply_block(typename Tr<P>::acc (&bot)[NB / 16], typename Tr<P>::S *top, int b,
                        const typename Tr<P>::S *Ys, const typename Tr<P>::S *Ts) {
    typedef typename Tr<P>::S S;
    typedef typename Tr<P>::acc acc_t;
    constexpr int LDY = qr_ldy<NB>();
    constexpr int P2 = (P == P64) ? P64 : P32;  // precision of the small T^T W product
    constexpr int NQ = IB / 16;                 // 16-reflector groups of the block
    constexpr int RB = NB / 16;
    static_assert(NQ == 1 || NQ == 2, "IB is 16 or 32");
    const int l = lane_id(), g = l >> 4, i16 = l & 15;
    const S *Yc = Ys, *Yr = vrow<NB>(Ys);
    // lane (i16, g) needs V(16 rb + drow(g, r), 16 qb + i16) in the W phase and
    // V(16 rb + i16, 16 ob + drow(g, r)) in the update; for 4-byte storage
    // (drow = 4g + r) both are one 128-bit read per (block, rb)
    auto vw = [&](int qb, int rb) { return *(const f4 *)&Yc[(16 * qb + i16) * LDY + 16 * rb + 4 * g]; };
    auto vu = [&](int ob, int rb) { return *(const f4 *)&Yr[(16 * rb + i16) * LDQ + 16 * ob + 4 * g]; };
    S tv[NQ][4];
    if constexpr (HAS_TOP) {
#pragma unroll
        for (int h = 0; h < NQ; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) tv[h][r] = top[IB * b + 16 * h + Tr<P>::drow(g, r)];
    }
    acc_t Wc[2][NQ];
#pragma unroll
    for (int h = 0; h < NQ; ++h) Wc[0][h] = Wc[1][h] = zero_acc<acc_t>();
    f4 va[NQ][RB], ua[NQ][RB];
    if constexpr (P == P32 && PRE) {
#pragma unroll
        for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) va[qb][rb] = vw(qb, rb);
#pragma unroll
        for (int ob = 0; ob < NQ; ++ob)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) ua[ob][rb] = vu(ob, rb);
        __builtin_amdgcn_sched_barrier(0);
    }
    // W += V^T bot
    if constexpr (P == P32) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int qb = 0; qb < NQ; ++qb) {
                const f4 y = PRE ? va[qb][rb] : vw(qb, rb);
#pragma unroll
                for (int r = 0; r < 4; ++r) Wc[rb & 1][qb] = Tr<P>::mma(y[r], bot[rb][r], Wc[rb & 1][qb]);
            }
    } else if constexpr (P == P64) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int qb = 0; qb < NQ; ++qb)
                    Wc[rb & 1][qb] = Tr<P>::mma(Yc[(16 * qb + i16) * LDY + 16 * rb + Tr<P>::drow(g, r)], bot[rb][r],
                                                Wc[rb & 1][qb]);
    } else {
#pragma unroll
        // three-term split: x = hi + lo with hi, lo in BF16, and the product
        // as hi.hi + hi.lo + lo.hi (the dropped lo.lo term is 2^-16 relative):
        // every block application would otherwise perturb the tile by the
        // BF16 rounding of its operands, and a tile receives one per block
        // of every panel tile below it
        for (int pr = 0; pr < NB / 32; ++pr) {
            bf8 bh, bl;
#pragma unroll
            for (int e = 0; e < 8; ++e) { const float xs_ = bot[2 * pr + (e >> 2)][e & 3]; bh[e] = bf_hi(xs_); bl[e] = bf_lo(xs_); }
#pragma unroll
            for (int qb = 0; qb < NQ; ++qb) {
                const f4 v0 = vw(qb, 2 * pr), v1 = vw(qb, 2 * pr + 1);
                bf8 ah, al;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    { const float xs_ = v0[e]; ah[e] = bf_hi(xs_); al[e] = bf_lo(xs_); }
                    { const float xs_ = v1[e]; ah[4 + e] = bf_hi(xs_); al[4 + e] = bf_lo(xs_); }
                }
                Wc[pr & 1][qb] = Tr<PB16>::mma(ah, bh, Wc[pr & 1][qb]);
                Wc[pr & 1][qb] = Tr<PB16>::mma(ah, bl, Wc[pr & 1][qb]);
                Wc[pr & 1][qb] = Tr<PB16>::mma(al, bh, Wc[pr & 1][qb]);
            }
        }
    }
    acc_t Wb[NQ];
#pragma unroll
    for (int h = 0; h < NQ; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Wb[h][r] = Wc[0][h][r] + Wc[1][h][r];
            if constexpr (HAS_TOP) Wb[h][r] += tv[h][r];
        }
    // W' = T^T W
    acc_t Wp[NQ];
#pragma unroll
    for (int ob = 0; ob < NQ; ++ob) Wp[ob] = zero_acc<acc_t>();
#pragma unroll
    for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int ob = 0; ob < NQ; ++ob)
                Wp[ob] = Tr<P2>::mma(Ts[(16 * ob + i16) * IB + 16 * qb + Tr<P>::drow(g, r)], Wb[qb][r], Wp[ob]);
    if constexpr (HAS_TOP) {
#pragma unroll
        for (int h = 0; h < NQ; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) top[IB * b + 16 * h + Tr<P>::drow(g, r)] = (S)(tv[h][r] - Wp[h][r]);
    }
    // bot -= V W', as bot += V (-W'): the sign goes on the NQ x 4 values of W'
    // once rather than on each of the V operands
#pragma unroll
    for (int ob = 0; ob < NQ; ++ob) Wp[ob] = -Wp[ob];
    if constexpr (P == P32) {
#pragma unroll
        for (int ob = 0; ob < NQ; ++ob)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const f4 y = PRE ? ua[ob][rb] : vu(ob, rb);
#pragma unroll
                for (int r = 0; r < 4; ++r) bot[rb] = Tr<P>::mma(y[r], Wp[ob][r], bot[rb]);
            }
    } else if constexpr (P == P64) {
#pragma unroll
        for (int ob = 0; ob < NQ; ++ob)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    bot[rb] = Tr<P>::mma(Yr[(16 * rb + i16) * LDQ + 16 * ob + Tr<P>::drow(g, r)], Wp[ob][r], bot[rb]);
    } else {
        // K = 32 per MFMA (a 16-reflector block fills the second half with
        // zeros); the same three-term split as above
        bf8 wh, wl;
#pragma unroll
        for (int e = 0; e < 8; ++e) { const float xs_ = (e >> 2) < NQ ? Wp[(e >> 2) % NQ][e & 3] : 0.0f; wh[e] = bf_hi(xs_); wl[e] = bf_lo(xs_); }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            bf8 ah, al;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                f4 v = {0.0f, 0.0f, 0.0f, 0.0f};
                if (h < NQ) v = vu(h, rb);
#pragma unroll
                for (int e = 0; e < 4; ++e) { const float xs_ = v[e]; ah[4 * h + e] = bf_hi(xs_); al[4 * h + e] = bf_lo(xs_); }
            }
            bot[rb] = Tr<PB16>::mma(ah, wh, bot[rb]);
            bot[rb] = Tr<PB16>::mma(ah, wl, bot[rb]);
            bot[rb] = Tr<PB16>::mma(al, wh, bot[rb]);
        }
    }
}

// Staging of block reflector b of tile V (column block c0 = b*IB) and its T
// block for apply_block, in two halves so that the global loads of the next
// block can be in flight while the current one is applied:
//   stage_load:  V(:, c0..c0+IB) and T(c0.., c0..) into registers;
//   stage_store: into LDS, both copies of V(:, c0..c0+IB) and Ts[q*IB + p] = T(p, q);
//                VM selects how V is held in the tile (below).
template <int NB, class S> struct StageRegs {
    static constexpr int PY = NB * IB / WG, PT = IB * IB / WG;
    static_assert(PY * WG == NB * IB && PT * WG == IB * IB, "whole elements per thread");
    S y[PY], t[PT];
};

template <int NB, class S>
LQ_DEV void stage_load(const S *V, const S *T, int c0, StageRegs<NB, S> &sr) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < StageRegs<NB, S>::PY; ++u) {
        const int e = tid + WG * u, r = e % NB, q = e / NB;
        sr.y[u] = V[r + (size_t)(c0 + q) * NB];
    }
#pragma unroll
    for (int u = 0; u < StageRegs<NB, S>::PT; ++u) {
        const int e = tid + WG * u;
        sr.t[u] = T[(c0 + e % IB) + (size_t)(c0 + e / IB) * NB];
    }
}

// VM: how V is held in the tile: 0 (TS) as stored; 1 (GEQRT) unit lower,
// zeros above and ones on the diagonal made explicit; 2 (TT) upper triangular,
// the entries below the diagonal (another reflector set) read as zeros.
template <int NB, class S, int VM>
LQ_DEV void stage_store(const StageRegs<NB, S> &sr, int c0, S *Ys, S *Ts) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < StageRegs<NB, S>::PY; ++u) {
        const int e = tid + WG * u, r = e % NB, q = e / NB;
        S v = sr.y[u];
        if (VM == 1) v = r < c0 + q ? (S)0 : (r == c0 + q ? (S)1 : v);
        if (VM == 2) v = r <= c0 + q ? v : (S)0;
        put_v<NB>(Ys, r, q, v);
    }
#pragma unroll
    for (int u = 0; u < StageRegs<NB, S>::PT; ++u) {
        const int e = tid + WG * u;
        Ts[(e / IB) * IB + e % IB] = sr.t[u];
    }
}

template <int NB, class S, int VM>
LQ_DEV void stage_block(const S *V, const S *T, int c0, S *Ys, S *Ts) {
    StageRegs<NB, S> sr;
    stage_load<NB, S>(V, T, c0, sr);
    stage_store<NB, S, VM>(sr, c0, Ys, Ts);
}

// Trailing update of a producer panel: columns (b+1)*IB..NB-1 of A (and, for
// TS, rows b*IB..b*IB+IB of R) in 64-column strips, with the consumer routine.
template <int NB, int P, bool TS, bool PRE = true, bool TT = false>
LQ_DEV void panel_trailing(typename Tr<P>::S *A, typename Tr<P>::S *R, int b, const typename Tr<P>::S *Ys,
                           const typename Tr<P>::S *Ts) {
    typedef typename Tr<P>::S S;
    typedef typename Tr<P>::acc acc_t;
    const int l = lane_id(), w = wave_id(), g = l >> 4, i16 = l & 15;
    for (int s0 = (b + 1) * IB; s0 < NB; s0 += 64) {
        const int col = s0 + 16 * w;
        if (col >= NB) continue;
        acc_t bot[NB / 16];
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + Tr<P>::drow(g, r);
                bot[rb][r] = (!TT || row <= col + i16) ? A[row + (col + i16) * NB] : (S)0;  // TT: upper part only
            }
        apply_block<NB, P, TS, PRE>(bot, TS ? R + (col + i16) * NB : nullptr, b, Ys, Ts);
        // GEQRT: rows above the block are untouched by its reflectors and belong
        // to R row blocks other producers are updating: write back rows >= c0 only
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + Tr<P>::drow(g, r);
                if ((TS || row >= b * IB) && (!TT || row <= col + i16)) A[row + (col + i16) * NB] = (S)bot[rb][r];
            }
    }
}

template <int NB, int P> constexpr int qr_lds() {
    return (qr_vblk<NB>() + 2 * IB * IB) * (int)sizeof(typename Tr<P>::S) + (int)sizeof(PanelLds);
}

// Consumer strips of 64 columns (16 per wave); for nb = 32 one strip with two
// active waves.
template <int NB> constexpr int qr_spc() { return NB >= 64 ? NB / 64 : 1; }

template <int NB> constexpr int qr_pw() { return NB / IB; }  // producer workgroups

LQ_DEV int *qr_flag(const Ctx &c, int i, int b) { return &c.flags[(size_t)i * (c.nb / IB) + b]; }

// One chain of a QR-step launch: the top tile row eliminates tile rows
// mfirst..end-1 of tile column k in order, with TS kernels (Alg. 4a), or, for
// a killed head of the elimination tree, with TT kernels on its upper
// triangle (tt; Alg. 4b).  geqrt: the top tile is factored first (GEQRT) and
// its own row gets the UNMQR blocks.  Launch 0 of a step holds one chain per
// group of the tree (the whole panel for the flat tree), launch d (d = 1, 2,
// 4, ..) one per pair of heads at distance d; flags carry the launch's epoch.
struct QrChain {
    int top, mfirst, end, epoch;
    bool geqrt, tt;
};

LQ_DEV QrChain qr_chain(const Ctx &c, int k, int d, int idx) {
    const QrTree tr(c.n, k, c.qtree);
    QrChain ch;
    if (d == 0) {
        ch.top = tr.head(idx); ch.mfirst = ch.top + 1; ch.end = tr.end(idx);
        ch.geqrt = true; ch.tt = false; ch.epoch = qr_epoch(k, 0);
    } else {
        const int g0 = 2 * d * idx;
        ch.top = tr.head(g0); ch.mfirst = tr.head(g0 + d); ch.end = ch.mfirst + 1;
        ch.geqrt = false; ch.tt = true; ch.epoch = qr_epoch(k, QrTree::level(d));
    }
    return ch;
}

// Variant A2 (Sec. 2.3) factors A_kk in its panel, before the decision
// (k_a2_geqrt, which publishes the flags of tile k); a QR step then continues
// from it (QR_REST: the producers of the chain topped by tile k skip its GEQRT
// unit, its consumers still apply the UNMQR blocks).
enum QrMode { QR_FULL = 0, QR_REST = 1 };

// Producer workgroup b of one chain: block b of GEQRT(top) (unless skipped),
// then block b of each TSQRT/TTQRT(top, A_ik) in order of i.  Unit (i, b)
// needs the trailing update of unit (i, b-1) (flag) and R's row block b (its
// own previous unit).  akk, tkk: where the GEQRT unit works instead of the
// top tile and its T factor (the A2 panel's FP64 copy).
template <int NB, int P, bool PRE, bool TT>
LQ_DEV void qr_producer(const Ctx &c, int k, const QrChain &ch, int b, char *smem, bool skip_geqrt,
                        typename Tr<P>::S *akk = nullptr, typename Tr<P>::S *tkk = nullptr) {
    typedef typename Tr<P>::S S;
    constexpr int PP = (P == PB16) ? P32 : P;  // panel-internal updates stay in the storage precision
    S *Ys = (S *)smem;
    S *Ts = Ys + qr_vblk<NB>();
    S *Rb = Ts + IB * IB;
    PanelLds *pl = (PanelLds *)(Rb + IB * IB);
    __shared__ int bail;
    S *At = (S *)c.At;
    S *Tq = (S *)(TT ? c.Tt : c.Tf);
    const int tid = threadIdx.x;
    const int epoch = ch.epoch;
    const int c0 = b * IB;
    S *Akk = akk ? akk : At + c.toff(ch.top, k);
    for (int i = (ch.geqrt && !skip_geqrt) ? ch.top : ch.mfirst; i < ch.end; ++i) {
        if (b > 0) {  // the trailing update of unit (i, b-1) must be in place
            if (tid == 0) bail = !flag_wait(qr_flag(c, i, b - 1), epoch, &c.st->watchdog);
            __syncthreads();
            if (bail) return;
            fence_acquire();
        }
        S *Ti = (i == ch.top && tkk) ? tkk : Tq + c.tqoff(i, k);
        if (i == ch.top) {
            panel_qr<NB, S, false>(Akk, c0, nullptr, Ys, Ts, pl);
            for (int e = tid; e < IB * IB; e += WG) Ti[(c0 + e % IB) + (c0 + e / IB) * NB] = Ts[e];
            panel_trailing<NB, PP, false, PRE>(Akk, nullptr, b, Ys, Ts);
        } else {
            S *Aik = At + c.toff(i, k);
            for (int e = tid; e < IB * IB; e += WG) {  // Rb row-major: Rb[p*IB + q] = R(p, q)
                const int p = e / IB, q = e % IB;
                Rb[e] = p <= q ? Akk[(c0 + p) + (c0 + q) * NB] : (S)0;
            }
            __syncthreads();
            panel_qr<NB, S, true, TT>(Aik, c0, Rb, Ys, Ts, pl);
            for (int e = tid; e < IB * IB; e += WG) {
                const int p = e % IB, q = e / IB;
                if (p <= q) Akk[(c0 + p) + (c0 + q) * NB] = Rb[p * IB + q];
                Ti[(c0 + p) + (c0 + q) * NB] = Ts[e];
            }
            panel_trailing<NB, PP, true, PRE, TT>(Aik, Akk, b, Ys, Ts);
        }
        fence_release();  // every thread's writes of unit (i, b) before the flag
        __syncthreads();
        if (tid == 0) flag_publish(qr_flag(c, i, b), epoch);
    }
}

// Consumer LDS: two staging buffers (block s is applied from one while block
// s+1 is written into the other).  When they and the producer's panel fit in
// half the LDS (4-byte storage, nb <= 256) the kernel is built for two
// workgroups per CU: then every workgroup of the widest steps is resident at
// once, and one workgroup's barriers, flag waits and staging overlap the
// other's MFMAs.  Otherwise (FP64, nb = 512) one workgroup per CU.
template <int NB, int P> constexpr int qr_stage_lds() {
    return 2 * (qr_vblk<NB>() + IB * IB) * (int)sizeof(typename Tr<P>::S);
}
template <int NB, int P> constexpr int qr_step_lds() {
    return qr_lds<NB, P>() > qr_stage_lds<NB, P>() ? qr_lds<NB, P>() : qr_stage_lds<NB, P>();
}
template <int NB, int P> constexpr int qr_occ() { return qr_step_lds<NB, P>() <= 80 * 1024 ? 2 : 1; }

// Launch d of QR step k (d = 0: the groups' chains, TT = false; d > 0: the TT
// level at distance d, TT = true): the chains' producers first (nb/IB
// workgroups per chain, so they are dispatched before any consumer and a
// consumer never waits on an unscheduled producer), then per chain one
// consumer per 64-column strip of every trailing tile column.
// Keepers (a single chain, two workgroups per CU, a grid that doubles up at
// least 2 nb/IB CUs but still fits at two per CU): the workgroups numbered
// QR_CUS + b.  Dispatch in order fills every CU once before it doubles any,
// so on an otherwise idle GPU workgroup QR_CUS + b lands beside producer b.
// The keeper only waits for that producer's last unit, which keeps the
// producer's CU for it: a consumer beside it slows the producer, and the
// producer chain paces every consumer.  The consumers it displaces double up
// with other consumers, so it pays only once enough of them do anyway
// (measured: slower at 16 doubled workgroups, faster from about 40).  (If
// keepers land elsewhere, they only wait.)  Their number in the groups'
// launch (d = 0) of step k (0 or nb/IB):
constexpr int QR_CUS = 256;
template <int NB, int P> LQ_HD int qr_keepers(int64_t n, int k, int nch) {
    const int all = qr_pw<NB>() + ((int)n - k - 1) * qr_spc<NB>();
    return (qr_occ<NB, P>() == 2 && nch == 1 && all >= QR_CUS + 2 * qr_pw<NB>() &&
            all + qr_pw<NB>() <= 2 * QR_CUS)
               ? qr_pw<NB>()
               : 0;
}

// sig (flat tree, d = 0): each consumer of tile column k+1 adds one to
// eflag[k] once it has written its strip of tile (k+1, k+1), which no later
// block of the step touches, so that the GEPP of step k+1's panel can start
// on that tile while the rest of the step runs (qr_spc strips in all).
// smem: qr_step_lds bytes.
template <int NB, int P, bool TT>
LQ_DEV void qr_step_body(const Ctx &c, int k, int mode, int d, int sig, char *smem) {
    typedef typename Tr<P>::S S;
    typedef typename Tr<P>::acc acc_t;
    constexpr int VB = qr_vblk<NB>();
    constexpr int NBLK = NB / IB;
    constexpr bool PRE = false;  // bulk operand loads would exceed the registers at nb >= 256
    const QrTree tr(c.n, k, c.qtree);
    const int nch = d == 0 ? tr.G : tr.npairs(d);
    const int cps = ((int)c.n - k - 1) * qr_spc<NB>();  // consumers per chain
    if ((int)blockIdx.x < nch * qr_pw<NB>()) {
        const int idx = (int)blockIdx.x / qr_pw<NB>();
        qr_producer<NB, P, PRE, TT>(c, k, qr_chain(c, k, d, idx), (int)blockIdx.x % qr_pw<NB>(), smem,
                                    mode == QR_REST && d == 0 && idx == 0);
        return;
    }
    if (cps == 0) return;
    int cidx = (int)blockIdx.x - nch * qr_pw<NB>();
    const int nkeep = d == 0 ? qr_keepers<NB, P>(c.n, k, nch) : 0;  // as the host sized the groups' launch
    if (nkeep > 0 && (int)blockIdx.x >= QR_CUS) {
        const int b = (int)blockIdx.x - QR_CUS;
        if (b < nkeep) {  // a keeper: wait for producer b's last unit
            if (threadIdx.x == 0) {
                const QrChain ch = qr_chain(c, k, d, 0);
                (void)flag_wait(qr_flag(c, ch.end - 1, b), ch.epoch, &c.st->watchdog);
            }
            return;
        }
        cidx -= nkeep;
    }
    const QrChain ch = qr_chain(c, k, d, cidx / cps);
    // Consumer: one 64-column strip of trailing tile column j.  The blocks it
    // applies form one sequence s = 0 .. nblocks-1: block b of tile i = t0 +
    // s/NBLK, first (geqrt) the UNMQR blocks of the top tile on its own strip
    // A_top,j, then the TSMQR (TTMQR) blocks of every A_ik on (A_top,j, A_ij).  Block s+1 is
    // loaded into registers before block s is applied and stored into the
    // other LDS buffer afterwards, so each block costs one barrier.
    // Cache invalidation is the expensive half of acquiring a block (several
    // microseconds per wave), so one invalidation covers every block whose
    // flag was seen set before it: the wavefront order of the producers makes
    // flag (i', b') imply all flags (i <= i', b <= b'), so when the flag of
    // the last block of a tile is already set the whole tile is covered.
    // Thread 0 keeps the index `covered` up to which blocks are acquired; the
    // flag that would extend it is read early and waited on only if unset.
    S *At = (S *)c.At;
    S *Tq = (S *)(TT ? c.Tt : c.Tf);
    const int epoch = ch.epoch;
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    const int strip = cidx % cps;
    const int j = k + 1 + strip / qr_spc<NB>();
    const int col0 = (strip % qr_spc<NB>()) * 64 + 16 * w;
    const bool active = col0 < NB;
    const int g = l >> 4, i16 = l & 15;
    S *const Y0 = (S *)smem;          // staging buffer u: V at Y0 + u*VB, T at T0 + u*IB*IB
    S *const T0 = Y0 + 2 * VB;
    __shared__ int bail[2], inval[2];  // for block x: slot x & 1
    S *Akj = At + c.toff(ch.top, j);
    S *const topc = Akj + (col0 + i16) * NB;  // this lane's column of A_top,j for the TSMQR blocks
    const int t0 = ch.geqrt ? ch.top : ch.mfirst;
    const int nblocks = (ch.end - t0) * NBLK;
    const int spub = (sig && !TT && ch.top == k && j == k + 1) ? (k + 1 - t0) * NBLK + NBLK - 1 : -1;
    auto vtile = [&](int s) { return At + c.toff(t0 + s / NBLK, k); };
    auto ttile = [&](int s) { return Tq + c.tqoff(t0 + s / NBLK, k); };
    auto flag_of = [&](int s) { return qr_flag(c, t0 + s / NBLK, s % NBLK); };
    acc_t bot[NB / 16];
    auto load_bot = [&](const S *src) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) bot[rb][r] = src[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB];
    };
    auto store_bot = [&](S *dst) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB] = (S)bot[rb][r];
    };
    auto tile_end = [&](int s) { return (s / NBLK) * NBLK + NBLK - 1; };
    int covered = 1;  // thread 0: blocks 0..covered are acquired
    // prologue: block 0 staged, flag of block 1 awaited (nblocks >= 2 NBLK)
    if (tid == 0) {
        bail[0] = !flag_wait(flag_of(0), epoch, &c.st->watchdog);
        bail[1] = !flag_wait(flag_of(1), epoch, &c.st->watchdog);
        if (__hip_atomic_load(flag_of(NBLK - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch)
            covered = NBLK - 1;
        inval[0] = inval[1] = 0;
    }
    __syncthreads();
    if (bail[0] || bail[1]) return;
    fence_acquire();
    if (active) load_bot(At + c.toff(t0, j));
    stage_block<NB, S, TT ? 2 : 1>(vtile(0), ttile(0), 0, Y0, T0);  // a TT chain has no GEQRT tile
    __syncthreads();
    for (int s = 0; s < nblocks; ++s) {
        const int cur = s & 1;
        const bool has_next = s + 1 < nblocks;
        if (has_next && bail[(s + 1) & 1]) return;  // the flag of block s+1 was never set
        const int i = t0 + s / NBLK, b = s % NBLK;
        StageRegs<NB, S> nx;
        if (has_next) {
            if (inval[(s + 1) & 1]) cache_invalidate();
            stage_load<NB, S>(vtile(s + 1), ttile(s + 1), ((s + 1) % NBLK) * IB, nx);
        }
        // the flag of the last block of block s+2's tile: every lane reads it
        // (one cache line per wave, no branch), so the value is waited for only
        // where thread 0 tests it after the apply
        const int fe = __hip_atomic_load(flag_of(tile_end(s + 2 < nblocks ? s + 2 : s)), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        if (active) {
            const S *Yc = Y0 + cur * VB, *Tc = T0 + cur * (IB * IB);
            if (!TT && i == ch.top) apply_block<NB, P, false, PRE>(bot, nullptr, b, Yc, Tc);
            else apply_block<NB, P, true, PRE>(bot, topc, b, Yc, Tc);
            if (b == NBLK - 1) {  // tile i done: write it back, start on the next
                store_bot(i == ch.top ? Akj : At + c.toff(i, j));
                if (i + 1 < ch.end) load_bot(At + c.toff(i + 1, j));
            }
        }
        if (s == spub) fence_release();  // this strip of tile (k+1, k+1) before the count
        if (has_next) {
            S *Yn = Y0 + (cur ^ 1) * VB, *Tn = T0 + (cur ^ 1) * (IB * IB);
            if constexpr (TT) stage_store<NB, S, 2>(nx, ((s + 1) % NBLK) * IB, Yn, Tn);
            else if ((s + 1) / NBLK == 0) stage_store<NB, S, 1>(nx, ((s + 1) % NBLK) * IB, Yn, Tn);
            else stage_store<NB, S, 0>(nx, ((s + 1) % NBLK) * IB, Yn, Tn);
        }
        if (tid == 0 && s + 2 < nblocks) {
            int bl = 0, inv = 0;
            if (s + 2 > covered) {
                inv = 1;
                if (fe >= epoch) {
                    covered = tile_end(s + 2);
                } else {
                    bl = !flag_wait(flag_of(s + 2), epoch, &c.st->watchdog);
                    covered = s + 2;
                }
            }
            bail[s & 1] = bl;
            inval[s & 1] = inv;
        }
        __syncthreads();
        if (s == spub && tid == 0) __hip_atomic_fetch_add(&c.eflag[k], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int NB, int P, bool TT>
__global__ __launch_bounds__(WG, (qr_occ<NB, P>())) void k_qr_step(Ctx c, int k, int mode, int d) {
    if (c.dec[k] != 0) return;
    __shared__ __attribute__((aligned(16))) char smem[qr_step_lds<NB, P>()];
    qr_step_body<NB, P, TT>(c, k, mode, d, 0, smem);
}

// ---------------------------------------------------------------------------
// Completion of the nb x nb compact-WY factors of a QR step's panel tiles
// (needed by the solve only).  With V = [V_0 .. V_{B-1}] split in IB-column
// blocks and Q = Q_0 Q_1 .. Q_{B-1}, Q_b = I - V_b T_b V_b^T, the product is
// I - V T V^T with T upper triangular, diagonal blocks T_b, and (Schreiber and
// Van Loan's block recurrence) for each b the block column above the diagonal
//     T(0:c, c:c+IB) = -T(0:c, 0:c) (V(:,0:c)^T V(:,c:c+IB)) T_b,   c = b IB.
// For the TS tiles V = [I; Y] and the identity parts of different columns do
// not overlap, so V(:,0:c)^T V(:,c:) = Y(:,0:c)^T Y(:,c:); for the GEQRT tile
// V is the unit-lower part of the factored diagonal tile.
// ---------------------------------------------------------------------------
// The Gram matrix is formed in GB x GB blocks (GB = 32, the smallest tile of
// the four-wave MFMA routine): every block (a, b) with a < b, and with IB < GB
// also the diagonal blocks, whose upper off-diagonal IB-blocks the recurrence
// reads.
constexpr int GB = 32;
static_assert(GB % IB == 0, "IB divides the Gram block");
template <int NB> constexpr int qr_npairs() {
    return IB < GB ? (NB / GB) * (NB / GB + 1) / 2 : (NB / GB) * (NB / GB - 1) / 2;
}

// Gram blocks G(a, b) = V_a^T V_b in FP64 (MFMA), one GB x GB block per
// workgroup; grid (pairs, n-k).
// tt = 0: every panel tile's own reflectors (GEQRT for the heads of the
// elimination tree, tile k alone in the flat tree; TS for the rest); tt = 1:
// the TT reflectors of the killed heads (upper triangular tails).
template <int NB, int P>
__global__ __launch_bounds__(WG) void k_qr_gram(Ctx c, int k, int tt) {
    if (c.dec[k] != 0) return;
    typedef typename Tr<P>::S S;
    __shared__ __attribute__((aligned(16))) char smem[mma_lds_bytes<P64, GB, GB, 16>()];
    int p = blockIdx.x, bb = IB < GB ? 0 : 1;  // column block bb holds pairs p = 0..bb (or 0..bb-1)
    while (p >= bb + (IB < GB)) { p -= bb + (IB < GB); ++bb; }
    const int a0 = p * GB, b0 = bb * GB;
    const int t = blockIdx.y, i = k + t;
    const bool head = QrTree(c.n, k, c.qtree).is_head(i);
    if (tt && (!head || i == k)) return;
    const S *V = (const S *)c.At + c.toff(i, k);
    auto v = [&](int r, int col) -> double {
        if (tt) return r <= col ? (double)V[r + (size_t)col * NB] : 0.0;
        if (!head) return (double)V[r + (size_t)col * NB];
        return r < col ? 0.0 : (r == col ? 1.0 : (double)V[r + (size_t)col * NB]);
    };
    Tr<P64>::acc acc[1][1];
    acc_zero<P64, GB, GB, 2, 2>(acc);
    wg_mma<P64, GB, GB, 2, 2, 16>(
        acc, NB, [&](int r, int kk) { return v(kk, a0 + r); }, [&](int kk, int cc) { return v(kk, b0 + cc); }, smem);
    double *G = c.gram + (size_t)t * NB * NB;
    acc_foreach<P64, GB, GB, 2, 2>(acc, [&](int r, int cc, double x) { G[(a0 + r) + (size_t)(b0 + cc) * NB] = x; });
}

// Off-diagonal blocks of T, block column by block column; one workgroup per
// panel tile, grid n-k.  FP64 arithmetic, storage precision result.
// For block column b (c0 = b IB): Y1 = T(0:c0, 0:c0) G(0:c0, c0:c0+IB), then
// T(0:c0, c0:c0+IB) = -Y1 T_b.  Y1 runs over 16-column chunks of T, each
// staged in LDS with coalesced loads (the strictly lower part, which the
// workspace does not hold, is masked to zero on staging); thread (a1, q)
// accumulates rows a1 + AS m of column q.
template <int NB, int P>
__global__ __launch_bounds__(WG) void k_qr_tfull(Ctx c, int k, int tt) {
    if (c.dec[k] != 0) return;
    if (tt) {  // the TT pass: the killed heads only
        const int i = k + (int)blockIdx.x;
        if (i == k || !QrTree(c.n, k, c.qtree).is_head(i)) return;
    }
    typedef typename Tr<P>::S S;
    constexpr int AS = WG / IB;         // row stride: thread tid takes rows tid/IB + AS m
    constexpr int MR = (NB - IB) / AS;  // rows a per thread at most
    constexpr int CH = 16;              // columns of T per staged chunk
    __shared__ double Tc[CH * (NB - IB)];  // chunk of T(0:c0, a2c..a2c+CH), [col][row]
    __shared__ double Gc[CH * IB];         // G(a2c..a2c+CH, c0..c0+IB), [row][q]
    __shared__ double Y1[(NB - IB) * IB];  // Y1[a*IB + p]
    __shared__ double Tb[IB * IB];
    const int t = blockIdx.x, i = k + t;
    S *T = (S *)(tt ? c.Tt : c.Tf) + c.tqoff(i, k);
    const double *G = c.gram + (size_t)t * NB * NB;
    const int tid = threadIdx.x, q = tid & (IB - 1), a1 = tid / IB;
    for (int b = 1; b < NB / IB; ++b) {
        const int c0 = b * IB;
        for (int e = tid; e < IB * IB; e += WG) {
            const int pp = e / IB, qq = e % IB;
            Tb[e] = pp <= qq ? (double)T[(c0 + pp) + (size_t)(c0 + qq) * NB] : 0.0;  // Tb[p*IB + q]
        }
        double acc[MR];
#pragma unroll
        for (int m = 0; m < MR; ++m) acc[m] = 0.0;
        for (int a2c = 0; a2c < c0; a2c += CH) {
            const int rows = a2c + CH;  // rows 0..a2c+CH-1 can be nonzero in these columns
            __syncthreads();             // previous chunk consumed
            for (int e = tid; e < CH * rows; e += WG) {
                const int r = e % rows, cc = e / rows, a2 = a2c + cc;
                Tc[cc * (NB - IB) + r] = r <= a2 ? (double)T[r + (size_t)a2 * NB] : 0.0;
            }
            for (int e = tid; e < CH * IB; e += WG) {
                const int rr = e / IB, qq = e % IB;
                Gc[e] = G[(a2c + rr) + (size_t)(c0 + qq) * NB];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int a = a1 + AS * m;
                if (a < rows) {
                    double s = 0.0;
#pragma unroll
                    for (int cc = 0; cc < CH; ++cc) s += Tc[cc * (NB - IB) + a] * Gc[cc * IB + q];
                    acc[m] += s;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int a = a1 + AS * m;
            if (a < c0) Y1[a * IB + q] = acc[m];
        }
        __syncthreads();
        for (int a = a1; a < c0; a += AS) {
            double s = 0.0;
            for (int pp = 0; pp <= q; ++pp) s += Y1[a * IB + pp] * Tb[pp * IB + q];
            T[a + (size_t)(c0 + q) * NB] = (S)(-s);
        }
        __syncthreads();  // this block column is written before the next reads it
    }
}

}  // namespace lq
