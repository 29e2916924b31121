// Workgroup-level MFMA contraction used by the LU-step kernels and the
// inverse-norm kernel: acc(BM x BN) += A(BM x K) * B(K x BN), operands staged
// through LDS in K-chunks of BK.  A and B are read through functors that
// return double (conversion to the MFMA operand type happens on staging), so
// the same routine serves tiles in FP64 / FP32 storage, FP64 triangular
// inverses and row-gathered (pivoted) operands.
#pragma once
#include "common.h"

namespace lq {

// Wave tile: WM x WN waves, each holding (BM/WM/16) x (BN/WN/16) accumulator blocks.
template <int P, int BM, int BN, int WM, int WN>
struct MmaShape {
    static constexpr int MB = BM / WM / 16;
    static constexpr int NBK = BN / WN / 16;
    static_assert(WM * WN == 4, "4 waves");
    static_assert(MB >= 1 && NBK >= 1, "wave tile at least 16x16");
    typedef typename Tr<P>::acc acc_t;
    typedef typename Tr<P>::C c_t;
    LQ_DEV static int row0() { return (wave_id() / WN) * (BM / WM); }
    LQ_DEV static int col0() { return (wave_id() % WN) * (BN / WN); }
};

// LDS bytes needed by wg_mma.
template <int P, int BM, int BN, int BK>
constexpr int mma_lds_bytes() { return (BM + 1 + BN + 1) * BK * (int)sizeof(typename Tr<P>::C); }

template <int P, int BM, int BN, int WM, int WN, int BK, class FA, class FB>
LQ_DEV void wg_mma(typename Tr<P>::acc (&acc)[BM / WM / 16][BN / WN / 16], int K, FA fa, FB fb, void *smem) {
    typedef MmaShape<P, BM, BN, WM, WN> Sh;
    typedef typename Tr<P>::C c_t;
    constexpr int KPL = Tr<P>::KPL;
    constexpr int KS = 4 * KPL;  // K per MFMA
    static_assert(BK % KS == 0, "BK multiple of the MFMA K");
    c_t *As = (c_t *)smem;                // [BK][BM+1]
    c_t *Bs = As + BK * (BM + 1);         // [BK][BN+1]
    const int l = lane_id();
    const int r0 = Sh::row0(), c0 = Sh::col0();
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int idx = threadIdx.x; idx < BM * BK; idx += WG) {
            int r = idx % BM, kk = idx / BM;
            As[kk * (BM + 1) + r] = cvt<c_t>(k0 + kk < K ? fa(r, k0 + kk) : 0.0);
        }
        for (int idx = threadIdx.x; idx < BN * BK; idx += WG) {
            int kk = idx % BK, c = idx / BK;
            Bs[kk * (BN + 1) + c] = cvt<c_t>(k0 + kk < K ? fb(k0 + kk, c) : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK / KS; ++ks) {
            typename Tr<P>::frag a[Sh::MB], b[Sh::NBK];
#pragma unroll
            for (int mb = 0; mb < Sh::MB; ++mb) {
                if constexpr (KPL == 1) {
                    a[mb] = As[(ks * KS + (l >> 4)) * (BM + 1) + r0 + 16 * mb + (l & 15)];
                } else {
#pragma unroll
                    for (int e = 0; e < KPL; ++e)
                        a[mb][e] = As[(ks * KS + KPL * (l >> 4) + e) * (BM + 1) + r0 + 16 * mb + (l & 15)];
                }
            }
#pragma unroll
            for (int nb = 0; nb < Sh::NBK; ++nb) {
                if constexpr (KPL == 1) {
                    b[nb] = Bs[(ks * KS + (l >> 4)) * (BN + 1) + c0 + 16 * nb + (l & 15)];
                } else {
#pragma unroll
                    for (int e = 0; e < KPL; ++e)
                        b[nb][e] = Bs[(ks * KS + KPL * (l >> 4) + e) * (BN + 1) + c0 + 16 * nb + (l & 15)];
                }
            }
#pragma unroll
            for (int mb = 0; mb < Sh::MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < Sh::NBK; ++nb) acc[mb][nb] = Tr<P>::mma(a[mb], b[nb], acc[mb][nb]);
        }
        __syncthreads();
    }
}

// Visit every element of a wave's accumulators: f(row, col, value) with
// row/col relative to the workgroup tile.
template <int P, int BM, int BN, int WM, int WN, class F>
LQ_DEV void acc_foreach(typename Tr<P>::acc (&acc)[BM / WM / 16][BN / WN / 16], F f) {
    typedef MmaShape<P, BM, BN, WM, WN> Sh;
    const int l = lane_id();
    const int r0 = Sh::row0(), c0 = Sh::col0();
#pragma unroll
    for (int mb = 0; mb < Sh::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < Sh::NBK; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                f(r0 + 16 * mb + Tr<P>::drow(l >> 4, r), c0 + 16 * nb + (l & 15), (double)acc[mb][nb][r]);
}

template <int P, int BM, int BN, int WM, int WN>
LQ_DEV void acc_zero(typename Tr<P>::acc (&acc)[BM / WM / 16][BN / WN / 16]) {
    typedef MmaShape<P, BM, BN, WM, WN> Sh;
#pragma unroll
    for (int mb = 0; mb < Sh::MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < Sh::NBK; ++nb) acc[mb][nb] = zero_acc<typename Tr<P>::acc>();
}

// wg_mma with BF16 operands split in two terms, x = hi + lo with hi = bf16(x)
// and lo = bf16(x - hi): acc += Ah Bh + Ah Bl + Al Bh.  The dropped Al Bl term
// and the rounding of lo leave a relative operand error near 2^-16 instead
// of 2^-8, at three times the MFMA work.  Other precisions take one pass.
template <int P, int BM, int BN, int WM, int WN, int BK, class FA, class FB>
LQ_DEV void wg_mma_split(typename Tr<P>::acc (&acc)[BM / WM / 16][BN / WN / 16], int K, FA fa, FB fb, void *smem) {
    if constexpr (P != PB16) {
        wg_mma<P, BM, BN, WM, WN, BK>(acc, K, fa, fb, smem);
    } else {
        auto hi = [](double x) { return (double)(float)(__bf16)(float)x; };
        auto ah = [&](int r, int k) { return hi(fa(r, k)); };
        auto bh = [&](int k, int c) { return hi(fb(k, c)); };
        auto al = [&](int r, int k) { const double x = fa(r, k); return x - hi(x); };
        auto bl = [&](int k, int c) { const double x = fb(k, c); return x - hi(x); };
        wg_mma<P, BM, BN, WM, WN, BK>(acc, K, ah, bh, smem);
        wg_mma<P, BM, BN, WM, WN, BK>(acc, K, ah, bl, smem);
        wg_mma<P, BM, BN, WM, WN, BK>(acc, K, al, bh, smem);
    }
}

}  // namespace lq
