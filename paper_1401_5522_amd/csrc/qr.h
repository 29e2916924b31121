// QR step with TS kernels and a flat reduction tree (Alg. 3 and 4a: the
// eliminator of every A_ik is A_kk), run only when the device-side decision
// of step k says QR.  One launch per step:
//   workgroup 0 (producer): GEQRT(A_kk), then TSQRT(R_kk, A_ik) for
//     i = k+1..n-1 in order, publishing flag[i] = k+1 after each;
//   workgroups 1.. (consumers): one 64-column strip of one trailing tile
//     column j; apply UNMQR to the strip of A_kj once GEQRT is published, then
//     TSMQR(i) on the strips of (A_kj, A_ij) as each TSQRT(i) is published.
// A consumer keeps both strips in MFMA accumulator registers (each wave owns
// 16 columns over all nb rows) for the whole chain, so A_kj never leaves the
// chip between the n-k-1 updates it receives.
// Reflectors use the LAPACK convention: beta = -sign(alpha)||x||, tau = 0
// when the tail is zero.  Compact-WY factors are kept per IB = 32 columns:
// block b of T(i,k) sits at rows b*IB.. of the nb x IB tile Tf(i,k).
#pragma once
#include "mma.h"

namespace lq {

template <class S> LQ_DEV S sq(S x) { return x * x; }

// Build the IB x IB compact-WY factor of the panel reflectors from their Gram
// matrix G(l,q) = v_l^T v_q (l < q): T(q,q) = tau_q,
// T(0:q,q) = -tau_q T(0:q,0:q) G(0:q,q).  One wave; G, T in LDS [q*IB + l].
template <class S>
LQ_DEV void build_t(const S *G, S *Ts, const S *tau) {
    const int l = lane_id();
    for (int q = 0; q < IB; ++q) {
        S v = 0;
        if (l < q) {
            for (int p = l; p < q; ++p) v += Ts[p * IB + l] * G[q * IB + p];
            v = -tau[q] * v;
        } else if (l == q) {
            v = tau[q];
        }
        if (l < IB) Ts[q * IB + l] = v;
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// Producer: GEQRT of A (nb x nb, in place: V below the diagonal, R on and
// above), T factors into Tt (nb x IB).
// ---------------------------------------------------------------------------
template <int NB, class S>
LQ_DEV void geqrt_tile(S *A, S *Tt, char *smem) {
    constexpr int LD = NB + 1;
    S *Pn = (S *)smem;          // panel [IB][LD]
    S *G = Pn + IB * LD;        // [IB*IB]
    S *Ts = G + IB * IB;        // [IB*IB]
    S *tau = Ts + IB * IB;      // [IB]
    S *Wc = tau + IB;           // [IB*33] chunk of W
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    for (int c0 = 0; c0 < NB; c0 += IB) {
        for (int e = tid; e < (NB - c0) * IB; e += WG) {
            int r = c0 + e % (NB - c0), q = e / (NB - c0);
            Pn[q * LD + r] = A[r + (c0 + q) * NB];
        }
        __syncthreads();
        if (w == 0) {
            for (int q = 0; q < IB; ++q) {
                const int col = c0 + q;
                S ss = 0;
                for (int r = col + 1 + l; r < NB; r += 64) ss += sq(Pn[q * LD + r]);
                ss = wave_sum(ss);
                const S alpha = Pn[q * LD + col];
                S t = 0;
                if (ss != (S)0) {
                    S nrm = sqrt(alpha * alpha + ss);
                    S beta = alpha >= (S)0 ? -nrm : nrm;
                    t = (beta - alpha) / beta;
                    S scal = (S)1 / (alpha - beta);
                    for (int r = col + 1 + l; r < NB; r += 64) Pn[q * LD + r] *= scal;
                    wave_sync();
                    if (l == 0) Pn[q * LD + col] = beta;
                }
                if (l == 0) tau[q] = t;
                wave_sync();
                if (t != (S)0) {
                    for (int j = q + 1; j < IB; ++j) {
                        S d = 0;
                        for (int r = col + 1 + l; r < NB; r += 64) d += Pn[q * LD + r] * Pn[j * LD + r];
                        d = wave_sum(d);
                        const S wv = t * (Pn[j * LD + col] + d);
                        for (int r = col + 1 + l; r < NB; r += 64) Pn[j * LD + r] -= Pn[q * LD + r] * wv;
                        wave_sync();
                        if (l == 0) Pn[j * LD + col] -= wv;
                        wave_sync();
                    }
                }
            }
        }
        __syncthreads();
        // Gram matrix of the block's reflectors: v_l = e_{c0+l} + tail below row c0+l
        for (int e = tid; e < IB * IB; e += WG) {
            int lq = e % IB, q = e / IB;
            S g = 0;
            if (lq < q) {
                g = Pn[lq * LD + c0 + q];
                for (int r = c0 + q + 1; r < NB; ++r) g += Pn[lq * LD + r] * Pn[q * LD + r];
            }
            G[q * IB + lq] = g;
        }
        __syncthreads();
        if (w == 0) build_t<S>(G, Ts, tau);
        __syncthreads();
        for (int e = tid; e < (NB - c0) * IB; e += WG) {
            int r = c0 + e % (NB - c0), q = e / (NB - c0);
            A[r + (c0 + q) * NB] = Pn[q * LD + r];
        }
        for (int e = tid; e < IB * IB; e += WG) {
            int p = e % IB, q = e / IB;
            Tt[(c0 + p) + q * NB] = Ts[q * IB + p];
        }
        // trailing columns: C <- (I - V T V^T)^T C, 32 columns at a time
        for (int j0 = c0 + IB; j0 < NB; j0 += 32) {
            __syncthreads();
            for (int e = tid; e < IB * 32; e += WG) {  // Wc = V^T C
                int lq = e % IB, jj = e / IB;
                const S *Cc = A + (j0 + jj) * NB;
                S s = Cc[c0 + lq];
                for (int r = c0 + lq + 1; r < NB; ++r) s += Pn[lq * LD + r] * Cc[r];
                Wc[jj * 33 + lq] = s;
            }
            __syncthreads();
            S w2[4];
            for (int u = 0; u < 4; ++u) {  // W2 = T^T Wc
                int e = tid + u * WG;
                int lq = e % IB, jj = e / IB;
                S s = 0;
                for (int p = 0; p <= lq; ++p) s += Ts[lq * IB + p] * Wc[jj * 33 + p];
                w2[u] = s;
            }
            __syncthreads();
            for (int u = 0; u < 4; ++u) {
                int e = tid + u * WG;
                Wc[(e / IB) * 33 + e % IB] = w2[u];
            }
            __syncthreads();
            for (int e = tid; e < (NB - c0) * 32; e += WG) {  // C -= V W2
                int r = c0 + e % (NB - c0), jj = e / (NB - c0);
                S s = 0;
                const int lmax = r - c0 < IB ? r - c0 : IB - 1;
                for (int lq = 0; lq <= lmax; ++lq) {
                    S v = (r == c0 + lq) ? (S)1 : Pn[lq * LD + r];
                    s += v * Wc[jj * 33 + lq];
                }
                A[r + (j0 + jj) * NB] -= s;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Producer: TSQRT of [R; A] (R = upper triangle of the nb x nb tile Rt,
// A = nb x nb tile): Y overwrites A, R is updated in place, T into Tt.
// ---------------------------------------------------------------------------
template <int NB, class S>
LQ_DEV void tsqrt_tile(S *Rt, S *A, S *Tt, char *smem) {
    constexpr int LD = NB + 1;
    S *Pn = (S *)smem;           // [IB][LD]
    S *G = Pn + IB * LD;
    S *Ts = G + IB * IB;
    S *tau = Ts + IB * IB;
    S *Wc = tau + IB;            // [32*33]
    S *Rb = Wc + 32 * 33;        // [IB*IB] diagonal block of R, Rb[q*IB + p] = R(c0+p, c0+q)
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    for (int c0 = 0; c0 < NB; c0 += IB) {
        for (int e = tid; e < NB * IB; e += WG) {
            int r = e % NB, q = e / NB;
            Pn[q * LD + r] = A[r + (c0 + q) * NB];
        }
        for (int e = tid; e < IB * IB; e += WG) {
            int p = e % IB, q = e / IB;
            Rb[q * IB + p] = p <= q ? Rt[(c0 + p) + (c0 + q) * NB] : (S)0;
        }
        __syncthreads();
        if (w == 0) {
            for (int q = 0; q < IB; ++q) {
                S ss = 0;
                for (int r = l; r < NB; r += 64) ss += sq(Pn[q * LD + r]);
                ss = wave_sum(ss);
                const S alpha = Rb[q * IB + q];
                S t = 0;
                if (ss != (S)0) {
                    S nrm = sqrt(alpha * alpha + ss);
                    S beta = alpha >= (S)0 ? -nrm : nrm;
                    t = (beta - alpha) / beta;
                    S scal = (S)1 / (alpha - beta);
                    for (int r = l; r < NB; r += 64) Pn[q * LD + r] *= scal;
                    wave_sync();
                    if (l == 0) Rb[q * IB + q] = beta;
                }
                if (l == 0) tau[q] = t;
                wave_sync();
                if (t != (S)0) {
                    for (int j = q + 1; j < IB; ++j) {
                        S d = 0;
                        for (int r = l; r < NB; r += 64) d += Pn[q * LD + r] * Pn[j * LD + r];
                        d = wave_sum(d);
                        const S wv = t * (Rb[j * IB + q] + d);
                        for (int r = l; r < NB; r += 64) Pn[j * LD + r] -= Pn[q * LD + r] * wv;
                        wave_sync();
                        if (l == 0) Rb[j * IB + q] -= wv;
                        wave_sync();
                    }
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < IB * IB; e += WG) {  // Gram of the Y parts (the e_c parts are orthonormal)
            int lq = e % IB, q = e / IB;
            S g = 0;
            if (lq < q)
                for (int r = 0; r < NB; ++r) g += Pn[lq * LD + r] * Pn[q * LD + r];
            G[q * IB + lq] = g;
        }
        __syncthreads();
        if (w == 0) build_t<S>(G, Ts, tau);
        __syncthreads();
        for (int e = tid; e < NB * IB; e += WG) {
            int r = e % NB, q = e / NB;
            A[r + (c0 + q) * NB] = Pn[q * LD + r];
        }
        for (int e = tid; e < IB * IB; e += WG) {
            int p = e % IB, q = e / IB;
            if (p <= q) Rt[(c0 + p) + (c0 + q) * NB] = Rb[q * IB + p];
            Tt[(c0 + p) + q * NB] = Ts[q * IB + p];
        }
        for (int j0 = c0 + IB; j0 < NB; j0 += 32) {
            __syncthreads();
            for (int e = tid; e < IB * 32; e += WG) {  // Wc = R(c0.., cols) + Y^T A(:, cols)
                int lq = e % IB, jj = e / IB;
                const S *Cc = A + (j0 + jj) * NB;
                S s = Rt[(c0 + lq) + (j0 + jj) * NB];
                for (int r = 0; r < NB; ++r) s += Pn[lq * LD + r] * Cc[r];
                Wc[jj * 33 + lq] = s;
            }
            __syncthreads();
            S w2[4];
            for (int u = 0; u < 4; ++u) {
                int e = tid + u * WG;
                int lq = e % IB, jj = e / IB;
                S s = 0;
                for (int p = 0; p <= lq; ++p) s += Ts[lq * IB + p] * Wc[jj * 33 + p];
                w2[u] = s;
            }
            __syncthreads();
            for (int u = 0; u < 4; ++u) {
                int e = tid + u * WG;
                int lq = e % IB, jj = e / IB;
                Wc[jj * 33 + lq] = w2[u];
                Rt[(c0 + lq) + (j0 + jj) * NB] -= w2[u];
            }
            __syncthreads();
            for (int e = tid; e < NB * 32; e += WG) {
                int r = e % NB, jj = e / NB;
                S s = 0;
#pragma unroll 8
                for (int lq = 0; lq < IB; ++lq) s += Pn[lq * LD + r] * Wc[jj * 33 + lq];
                A[r + (j0 + jj) * NB] -= s;
            }
        }
        __syncthreads();
    }
}

template <int NB, class S> constexpr int producer_lds() {
    return (IB * (NB + 1) + 3 * IB * IB + IB + 32 * 33) * (int)sizeof(S);
}

// ---------------------------------------------------------------------------
// Consumer: apply one block reflector (I - V T V^T)^T to a wave's 16-column
// slice.  `bot` holds all nb rows of the slice being eliminated into; when
// HAS_TOP, `top` holds the eliminator row tile and only its rows
// [c0, c0+IB) take part (TS structure: V = [E; Y]).  Without HAS_TOP the
// reflector lives entirely in `bot`'s rows (UNMQR; V given explicitly).
// Ys[q*LDY + r] = Y(r, q), Ts[q*IB + p] = T(p, q).
// ---------------------------------------------------------------------------
template <int NB, int P, bool HAS_TOP>
LQ_DEV void apply_block(typename Tr<P>::acc (&bot)[NB / 16], typename Tr<P>::acc (&top)[NB / 16], int b,
                        const typename Tr<P>::S *Ys, const typename Tr<P>::S *Ts) {
    typedef typename Tr<P>::S S;
    typedef typename Tr<P>::acc acc_t;
    constexpr int LDY = NB + 1;
    constexpr int P2 = (P == P64) ? P64 : P32;  // precision of the small T^T W product
    const int l = lane_id(), g = l >> 4, i16 = l & 15;
    acc_t Wb[2];
    if constexpr (HAS_TOP) { Wb[0] = top[2 * b]; Wb[1] = top[2 * b + 1]; }
    else { Wb[0] = zero_acc<acc_t>(); Wb[1] = zero_acc<acc_t>(); }
    // W += Y^T bot
    if constexpr (P != PB16) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rb + Tr<P>::drow(g, r);
#pragma unroll
                for (int qb = 0; qb < 2; ++qb)
                    Wb[qb] = Tr<P>::mma(Ys[(16 * qb + i16) * LDY + row], bot[rb][r], Wb[qb]);
            }
    } else {
#pragma unroll
        for (int pr = 0; pr < NB / 32; ++pr) {
            bf8 bo;
#pragma unroll
            for (int e = 0; e < 8; ++e) bo[e] = (__bf16)bot[2 * pr + (e >> 2)][e & 3];
#pragma unroll
            for (int qb = 0; qb < 2; ++qb) {
                bf8 a;
#pragma unroll
                for (int e = 0; e < 8; ++e) a[e] = (__bf16)Ys[(16 * qb + i16) * LDY + 32 * pr + 16 * (e >> 2) + Tr<P>::drow(g, e & 3)];
                Wb[qb] = Tr<PB16>::mma(a, bo, Wb[qb]);
            }
        }
    }
    // W' = T^T W
    acc_t Wp[2] = {zero_acc<acc_t>(), zero_acc<acc_t>()};
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
                Wp[ob] = Tr<P2>::mma(Ts[(16 * ob + i16) * IB + 16 * qb + Tr<P>::drow(g, r)], Wb[qb][r], Wp[ob]);
    if constexpr (HAS_TOP) {
        top[2 * b] -= Wp[0];
        top[2 * b + 1] -= Wp[1];
    }
    // bot -= Y W'
    if constexpr (P != PB16) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    bot[rb] = Tr<P>::mma(-Ys[(16 * ob + Tr<P>::drow(g, r)) * LDY + 16 * rb + i16], Wp[ob][r], bot[rb]);
    } else {
        bf8 bw;
#pragma unroll
        for (int e = 0; e < 8; ++e) bw[e] = (__bf16)Wp[e >> 2][e & 3];
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb) {
            bf8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = (__bf16)(-Ys[(16 * (e >> 2) + Tr<P>::drow(g, e & 3)) * LDY + 16 * rb + i16]);
            bot[rb] = Tr<PB16>::mma(a, bw, bot[rb]);
        }
    }
}

template <int NB, int P> constexpr int consumer_lds() {
    return (IB * (NB + 1) + IB * IB) * (int)sizeof(typename Tr<P>::S);
}

template <int NB, int P> constexpr int qr_lds() {
    return producer_lds<NB, typename Tr<P>::S>() > consumer_lds<NB, P>() ? producer_lds<NB, typename Tr<P>::S>()
                                                                        : consumer_lds<NB, P>();
}

// Strips of 64 columns (16 per wave); for nb = 32 one strip with two active waves.
template <int NB> constexpr int qr_spc() { return NB >= 64 ? NB / 64 : 1; }

template <int NB, int P>
__global__ __launch_bounds__(WG, 1) void k_qr_step(Ctx c, int k) {
    if (c.dec[k] != 0) return;
    typedef typename Tr<P>::S S;
    typedef typename Tr<P>::acc acc_t;
    constexpr int LDY = NB + 1;
    __shared__ __attribute__((aligned(16))) char smem[qr_lds<NB, P>()];
    S *At = (S *)c.At;
    S *Tf = (S *)c.Tf;
    const int epoch = k + 1;
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    if (blockIdx.x == 0) {
        S *Akk = At + c.toff(k, k);
        geqrt_tile<NB, S>(Akk, Tf + c.toff(k, k) / NB * IB, smem);
        __threadfence();
        __syncthreads();
        if (tid == 0) flag_publish(&c.flags[k], epoch);
        for (int i = k + 1; i < c.n; ++i) {
            tsqrt_tile<NB, S>(Akk, At + c.toff(i, k), Tf + c.toff(i, k) / NB * IB, smem);
            __threadfence();
            __syncthreads();
            if (tid == 0) flag_publish(&c.flags[i], epoch);
        }
        return;
    }
    const int strip = (int)blockIdx.x - 1;
    const int j = k + 1 + strip / qr_spc<NB>();
    const int col0 = (strip % qr_spc<NB>()) * 64 + 16 * w;
    const bool active = col0 < NB;
    S *Ys = (S *)smem;
    S *Ts = Ys + IB * LDY;
    acc_t top[NB / 16], bot[NB / 16];
    S *Akj = At + c.toff(k, j);
    const int g = l >> 4, i16 = l & 15;
    if (active) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) top[rb][r] = Akj[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB];
    }
    __shared__ int bail;
    if (tid == 0) bail = !flag_wait(&c.flags[k], epoch, &c.st->watchdog);
    __syncthreads();
    if (bail) return;
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    {  // UNMQR on the strip of A_kj: explicit V blocks of the GEQRT tile
        const S *V = At + c.toff(k, k);
        const S *T = Tf + c.toff(k, k) / NB * IB;
        for (int b = 0; b < NB / IB; ++b) {
            const int c0 = b * IB;
            for (int e = tid; e < NB * IB; e += WG) {
                int r = e % NB, q = e / NB;
                S v = r < c0 + q ? (S)0 : (r == c0 + q ? (S)1 : V[r + (c0 + q) * NB]);
                Ys[q * LDY + r] = v;
            }
            for (int e = tid; e < IB * IB; e += WG) Ts[(e / IB) * IB + e % IB] = T[(c0 + e % IB) + (e / IB) * NB];
            __syncthreads();
            if (active) apply_block<NB, P, false>(top, bot, b, Ys, Ts);
            __syncthreads();
        }
    }
    for (int i = k + 1; i < c.n; ++i) {
        if (tid == 0) bail = !flag_wait(&c.flags[i], epoch, &c.st->watchdog);
        __syncthreads();
        if (bail) return;
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        S *Aij = At + c.toff(i, j);
        const S *Y = At + c.toff(i, k);
        const S *T = Tf + c.toff(i, k) / NB * IB;
        if (active) {
#pragma unroll
            for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) bot[rb][r] = Aij[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB];
        }
        for (int b = 0; b < NB / IB; ++b) {
            const int c0 = b * IB;
            for (int e = tid; e < NB * IB; e += WG) {
                int r = e % NB, q = e / NB;
                Ys[q * LDY + r] = Y[r + (c0 + q) * NB];
            }
            for (int e = tid; e < IB * IB; e += WG) Ts[(e / IB) * IB + e % IB] = T[(c0 + e % IB) + (e / IB) * NB];
            __syncthreads();
            if (active) apply_block<NB, P, true>(bot, top, b, Ys, Ts);
            __syncthreads();
        }
        if (active) {
#pragma unroll
            for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) Aij[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB] = (S)bot[rb][r];
        }
    }
    if (active) {
#pragma unroll
        for (int rb = 0; rb < NB / 16; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) Akj[(16 * rb + Tr<P>::drow(g, r)) + (col0 + i16) * NB] = (S)top[rb][r];
    }
}

}  // namespace lq
