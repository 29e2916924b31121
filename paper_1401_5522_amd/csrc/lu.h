// LU step, variant A1 (Alg. 2), run only when the device-side decision of
// step k says LU:
//   Factor   A_kk <- L\U from the GETRF copy,
//   Eliminate A_ik <- A_ik U^{-1}      (i > k),
//   Apply     A_kj <- L^{-1} P A_kj    (j > k),
//   Update    A_ij <- A_ij - A_ik A_kj (i, j > k).
// Variant A2 (Sec. 2.3) runs the same kernels with U^{-1} = R_kk^{-1},
// L^{-1} = Q_kk^T and P = I from its GEQRT panel; its Factor is that GEQRT,
// already in the tile.
// Eliminate and Apply multiply by the explicit triangular inverses computed
// for the criterion, so all three are MFMA contractions; each in-place
// product is computed by a workgroup that owns whole rows (Eliminate) or
// whole columns (Apply) of the output, so it reads all of its input before
// writing.
#pragma once
#include "mma.h"

namespace lq {

// Rows per Eliminate workgroup / columns per Apply workgroup: the output
// block (RB x NB) holds 16K elements in registers.
template <int NB> constexpr int lu_rb() { return NB >= 128 ? 16384 / NB : NB; }
// Wave grid of the Eliminate block (RB x NB) and Apply block (NB x RB).
template <int NB> constexpr int lu_wn() { return NB >= 64 ? 4 : 2; }

template <int P> LQ_DEV float tile_scale(const Ctx &c, int64_t i, int64_t j) {
    if constexpr (P != PB16) return 1.0f;
    float mx = __uint_as_float(c.tmax[j * c.n + i]);
    if (!(mx > 0.0f) || !isfinite(mx)) return 1.0f;
    return ldexpf(1.0f, -ilogbf(mx));  // scaled max in [1, 2)
}

template <int NB, int P>
__global__ __launch_bounds__(WG) void k_lu_apply(Ctx c, int k) {
    if (c.dec[k] != 1) return;
    typedef typename Tr<P>::S S;
    constexpr int RB = lu_rb<NB>();
    constexpr int WN = lu_wn<NB>(), WM = 4 / WN;
    constexpr int BK = (P == PB16) ? 32 : 16;
    __shared__ __attribute__((aligned(16))) char smem[mma_lds_bytes<P, (RB > NB ? RB : NB), (RB > NB ? RB : NB), BK>()];
    __shared__ float wmax[WG / 64];
    const int rest = (int)c.n - k - 1;
    const int per_tile = NB / RB;
    int b = blockIdx.x;
    S *At = (S *)c.At;
    if (b == 0) {  // commit the factored copy (L\U) to the diagonal tile
        if (c.a2) return;  // variant A2: the tile already holds V\R of its GEQRT
        const double *W = c.W + (size_t)k * NB * NB;
        S *Akk = At + c.toff(k, k);
        for (int e = threadIdx.x; e < NB * NB; e += WG) Akk[e] = (S)W[e];
        return;
    }
    b -= 1;
    float lmx = 0.0f;
    if (b < rest * per_tile) {  // Eliminate: rows [r0, r0+RB) of A_ik times U^{-1}
        const int i = k + 1 + b / per_tile, r0 = (b % per_tile) * RB;
        S *X = At + c.toff(i, k);
        if (c.indom(k, i)) {  // a domain tile: its multipliers come from the domain's GEPP
            const int t = (i - k) / c.dstride;
            for (int e = threadIdx.x; e < RB * NB; e += WG) {
                const int r = r0 + e % RB, cc = e / RB;
                const S o = (S)c.WD[(size_t)t * NB + r + (size_t)cc * c.DR];
                X[r + cc * NB] = o;
                lmx = fmaxf(lmx, fabsf((float)o));
            }
            if constexpr (P == PB16) {
                for (int o = 32; o > 0; o >>= 1) lmx = fmaxf(lmx, __shfl_xor(lmx, o, 64));
                if (lane_id() == 0) atomicMax(&c.tmax[(size_t)k * c.n + i], __float_as_uint(lmx));
            }
            return;
        }
        const double *Ui = c.Dinv + (size_t)k * NB * NB;
        typename Tr<P>::acc acc[RB / WM / 16][NB / WN / 16];
        acc_zero<P, RB, NB, WM, WN>(acc);
        wg_mma_split<P, RB, NB, WM, WN, BK>(
            acc, NB, [&](int r, int kk) { return (double)X[r0 + r + kk * NB]; },
            [&](int kk, int cc) { return Ui[kk + (size_t)cc * NB]; }, smem);
        __syncthreads();
        acc_foreach<P, RB, NB, WM, WN>(acc, [&](int r, int cc, double v) {
            S o = (S)v;
            X[r0 + r + cc * NB] = o;
            lmx = fmaxf(lmx, fabsf((float)o));
        });
        if constexpr (P == PB16) {
            for (int o = 32; o > 0; o >>= 1) lmx = fmaxf(lmx, __shfl_xor(lmx, o, 64));
            if (lane_id() == 0) atomicMax(&c.tmax[(size_t)k * c.n + i], __float_as_uint(lmx));
        }
        return;
    }
    b -= rest * per_tile;
    {  // Apply: columns [c0, c0+RB) of A_kj <- L^{-1} (P A_kj)
        const int j = k + 1 + b / per_tile, c0 = (b % per_tile) * RB;
        S *X = At + c.toff(k, j);
        const double *Li = c.Linv + (size_t)k * NB * NB;
        const int *pm = c.perm + (size_t)k * NB;
        typename Tr<P>::acc acc[NB / WN / 16][RB / WM / 16];
        acc_zero<P, NB, RB, WN, WM>(acc);
        wg_mma_split<P, NB, RB, WN, WM, BK>(
            acc, NB, [&](int r, int kk) { return Li[r + (size_t)kk * NB]; },
            [&](int kk, int cc) { return (double)X[pm[kk] + (c0 + cc) * NB]; }, smem);
        __syncthreads();
        acc_foreach<P, NB, RB, WN, WM>(acc, [&](int r, int cc, double v) {
            S o = (S)v;
            X[r + (c0 + cc) * NB] = o;
            lmx = fmaxf(lmx, fabsf((float)o));
        });
        if constexpr (P == PB16) {
            for (int o = 32; o > 0; o >>= 1) lmx = fmaxf(lmx, __shfl_xor(lmx, o, 64));
            if (lane_id() == 0) atomicMax(&c.tmax[(size_t)j * c.n + k], __float_as_uint(lmx));
        }
    }
    (void)wmax;
}

// Diagonal domain, LU step: the trailing columns j > k of the domain's rows
// take the stacked permutation of its GEPP, (P D)(s,:) = D(dperm[s],:), so
// that Apply needs no interchanges of its own (Sec. 2.1: with this variant
// Apply works on the domain's interchanged rows).  Grid: (n-k-1) tile
// columns x NB/16 chunks of 16 columns; a workgroup gathers the domain rows
// of its chunk into LDS and writes back the rows that move.  BF16 tile maxima:
// rows only move among the domain's tiles of one column, so their largest
// maximum bounds each of them afterwards.
constexpr int DSW_CW = 16;  // columns per workgroup
template <int NB, int P>
__global__ __launch_bounds__(WG) void k_domain_swap(Ctx c, int k) {
    if (c.dec[k] != 1) return;
    const int d = c.dcount(k);
    if (d < 2) return;
    typedef typename Tr<P>::S S;
    __shared__ S buf[512 * DSW_CW];
    const int R = d * NB;
    const int j = k + 1 + (int)blockIdx.x / (NB / DSW_CW), c0 = ((int)blockIdx.x % (NB / DSW_CW)) * DSW_CW;
    const int *pm = c.dperm + (size_t)k * c.DR;
    S *At = (S *)c.At;
    auto at = [&](int sr, int cc) -> S * {
        return At + c.toff(k + (int64_t)(sr / NB) * c.dstride, j) + sr % NB + (size_t)(c0 + cc) * NB;
    };
    for (int e = threadIdx.x; e < R * DSW_CW; e += WG) buf[e] = *at(e % R, e / R);
    __syncthreads();
    for (int e = threadIdx.x; e < R * DSW_CW; e += WG) {
        const int r = e % R, sr = pm[r];
        if (sr != r) *at(r, e / R) = buf[sr + (e / R) * R];
    }
    if constexpr (P == PB16) {
        if (threadIdx.x == 0 && c0 == 0) {
            unsigned mx = 0;
            for (int t = 0; t < d; ++t) mx = max(mx, c.tmax[(size_t)j * c.n + k + (int64_t)t * c.dstride]);
            for (int t = 0; t < d; ++t) atomicMax(&c.tmax[(size_t)j * c.n + k + (int64_t)t * c.dstride], mx);
        }
    }
}

// Update: A_ij -= A_ik A_kj over the (n-k-1)^2 trailing tiles, BT x BT
// output blocks per workgroup.  BF16 mode: each tile is scaled by a power of
// two (its max |a| in [1,2)), the operands are split into bf16 hi + lo terms
// (wg_mma_split), the product accumulates in FP32 and is scaled back exactly.
template <int NB> constexpr int upd_bt() { return NB >= 128 ? 128 : NB; }

// FP32 storage, nb >= 128: a dedicated 128 x 128 x nb tile product.
//   * K runs in chunks of 32, staged in LDS K-contiguous: As[m][k] (A_ik is
//     column-major, so each thread transposes a 4 x 4 block in registers)
//     and Bs[n][k] (A_kj columns are K-contiguous already), row stride 36.
//   * Lane (i16, g) takes K index 16 G + 4 g + s in step s of group G, for A
//     and B alike, so each MFMA operand comes from one 128-bit LDS read that
//     serves four MFMAs; with stride 36 the sixteen lanes of a quarter-wave
//     hit sixteen disjoint bank groups.
//   * The next chunk is loaded into registers while the current one is
//     multiplied, then stored into the other LDS buffer: one barrier a chunk.
//   * Four waves of 64 x 64 (4 x 4 MFMA blocks of 16 x 16); the update of C
//     reads and writes four consecutive rows per lane (16 bytes), the reads
//     issued with the first chunk's loads.
// 74 KB of LDS and at most 256 registers: two workgroups per CU.
constexpr int UPD_BK = 32, UPD_LD = UPD_BK + 4;
constexpr int upd_lds_floats() { return 2 * 2 * 128 * UPD_LD; }

template <int NB>
LQ_DEV void lu_update_f32(const float *__restrict__ Aik, const float *__restrict__ Akj, float *__restrict__ C,
                          int r0, int c0, float *sm) {
    const int tid = threadIdx.x, l = lane_id(), w = wave_id(), g = l >> 4, i16 = l & 15;
    const int m0 = (w & 1) * 64, n0 = (w >> 1) * 64;  // the wave's 64 x 64 block
    // staging assignment: A: 4 rows (4 m4 ..) x 4 k (4 kq ..); B: row n = tid / 2, 16 k from 16 (tid & 1)
    const int m4 = tid & 31, kq = tid >> 5, bn = tid >> 1, bh = tid & 1;
    f4 ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[u] = *(const f4 *)&Aik[(r0 + 4 * m4) + (size_t)(k0 + 4 * kq + u) * NB];
#pragma unroll
        for (int u = 0; u < 4; ++u) rb[u] = *(const f4 *)&Akj[(k0 + 16 * bh + 4 * u) + (size_t)(c0 + bn) * NB];
    };
    auto store = [&](int buf) {
        float *As = sm + buf * (2 * 128 * UPD_LD), *Bs = As + 128 * UPD_LD;
#pragma unroll
        for (int i = 0; i < 4; ++i)  // row 4 m4 + i of the 4 x 4 block, k = 4 kq .. 4 kq + 3
            *(f4 *)&As[(4 * m4 + i) * UPD_LD + 4 * kq] = (f4){ra[0][i], ra[1][i], ra[2][i], ra[3][i]};
#pragma unroll
        for (int u = 0; u < 4; ++u) *(f4 *)&Bs[bn * UPD_LD + 16 * bh + 4 * u] = rb[u];
    };
    f4 acc[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    load(0);
    // this lane's part of C, loaded now so that the update at the end does not wait for it
    f4 cpre[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            cpre[mb][nb] = *(const f4 *)&C[(r0 + m0 + 16 * mb + 4 * g) + (size_t)(c0 + n0 + 16 * nb + i16) * NB];
    store(0);
    __syncthreads();
    constexpr int NCH = NB / UPD_BK;
    for (int ch = 0; ch < NCH; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < NCH) load((ch + 1) * UPD_BK);
        const float *As = sm + buf * (2 * 128 * UPD_LD), *Bs = As + 128 * UPD_LD;
#pragma unroll
        for (int G = 0; G < UPD_BK / 16; ++G) {
            f4 a[4], bv[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) a[mb] = *(const f4 *)&As[(m0 + 16 * mb + i16) * UPD_LD + 16 * G + 4 * g];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) bv[nb] = *(const f4 *)&Bs[(n0 + 16 * nb + i16) * UPD_LD + 16 * G + 4 * g];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mb][s], bv[nb][s], acc[mb][nb], 0, 0, 0);
        }
        if (ch + 1 < NCH) store(buf ^ 1);
        __syncthreads();
    }
    // C -= acc: lane (i16, g) owns rows 16 mb + 4 g .. + 3 of column 16 nb + i16
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
            *(f4 *)&C[(r0 + m0 + 16 * mb + 4 * g) + (size_t)(c0 + n0 + 16 * nb + i16) * NB] = cpre[mb][nb] - acc[mb][nb];
}

// FP64 storage, nb >= 128: the same 128 x 128 x nb tile product on
// v_mfma_f64_16x16x4f64.
//   * K runs in chunks of 16 doubles, staged K-contiguous with a row stride
//     of 18 doubles (144 bytes, so sixteen lanes' 16-byte reads hit sixteen
//     disjoint bank groups); A_ik is transposed through registers in 2 x 4
//     blocks, A_kj columns are K-contiguous already.
//   * Lane (i16, g) takes K index 8 G + 2 g + s in step s of group G for A and
//     B alike, so each operand pair comes from one 128-bit LDS read that
//     serves two MFMAs.
//   * Four waves of 64 x 64 (4 x 4 blocks of 16 x 16, 64 accumulator
//     doubles per lane); the next chunk is loaded into registers while the
//     current one is multiplied: one barrier a chunk.
// 74 KB of LDS and at most 256 registers: two workgroups per CU.
constexpr int UPD64_BK = 16, UPD64_LD = UPD64_BK + 2;
constexpr int upd64_lds_doubles() { return 2 * 2 * 128 * UPD64_LD; }

template <int NB>
LQ_DEV void lu_update_f64(const double *__restrict__ Aik, const double *__restrict__ Akj, double *__restrict__ C,
                          int r0, int c0, double *sm) {
    const int tid = threadIdx.x, l = lane_id(), w = wave_id(), g = l >> 4, i16 = l & 15;
    const int m0 = (w & 1) * 64, n0 = (w >> 1) * 64;  // the wave's 64 x 64 block
    // staging: A: rows 2 m2, 2 m2 + 1 at k = 4 kq .. 4 kq + 3; B: column n = tid / 2, k = 8 bh .. 8 bh + 7
    const int m2 = tid & 63, kq = tid >> 6, bn = tid >> 1, bh = tid & 1;
    d2 ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[u] = *(const d2 *)&Aik[(r0 + 2 * m2) + (size_t)(k0 + 4 * kq + u) * NB];
#pragma unroll
        for (int u = 0; u < 4; ++u) rb[u] = *(const d2 *)&Akj[(k0 + 8 * bh + 2 * u) + (size_t)(c0 + bn) * NB];
    };
    auto store = [&](int buf) {
        double *As = sm + buf * (2 * 128 * UPD64_LD), *Bs = As + 128 * UPD64_LD;
#pragma unroll
        for (int i = 0; i < 2; ++i) {  // row 2 m2 + i, k = 4 kq .. 4 kq + 3
            *(d2 *)&As[(2 * m2 + i) * UPD64_LD + 4 * kq] = (d2){ra[0][i], ra[1][i]};
            *(d2 *)&As[(2 * m2 + i) * UPD64_LD + 4 * kq + 2] = (d2){ra[2][i], ra[3][i]};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) *(d2 *)&Bs[bn * UPD64_LD + 8 * bh + 2 * u] = rb[u];
    };
    d4 acc[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = (d4){0.0, 0.0, 0.0, 0.0};
    load(0);
    store(0);
    __syncthreads();
    constexpr int NCH = NB / UPD64_BK;
    for (int ch = 0; ch < NCH; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < NCH) load((ch + 1) * UPD64_BK);
        const double *As = sm + buf * (2 * 128 * UPD64_LD), *Bs = As + 128 * UPD64_LD;
#pragma unroll
        for (int G = 0; G < UPD64_BK / 8; ++G) {
            d2 a[4], bv[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) a[mb] = *(const d2 *)&As[(m0 + 16 * mb + i16) * UPD64_LD + 8 * G + 2 * g];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) bv[nb] = *(const d2 *)&Bs[(n0 + 16 * nb + i16) * UPD64_LD + 8 * G + 2 * g];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][s], bv[nb][s], acc[mb][nb], 0, 0, 0);
        }
        if (ch + 1 < NCH) store(buf ^ 1);
        __syncthreads();
    }
    // C -= acc: lane (i16, g) owns rows 16 mb + g + 4 r of column 16 nb + i16
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *p = &C[(r0 + m0 + 16 * mb + Tr<P64>::drow(g, r)) + (size_t)(c0 + n0 + 16 * nb + i16) * NB];
                *p = *p - acc[mb][nb][r];
            }
}

template <int P> constexpr int upd_occ() { return P == P32 || P == P64 ? 2 : 1; }

// Tile columns j = jlo .. n-1 (grid: (n-k-1) (n-jlo) tiles x PER^2 blocks):
// jlo = k+1 for the whole update, or the lookahead column k+1 and the rest
// k+2.. as two launches.
template <int NB, int P>
__global__ __launch_bounds__(WG, (upd_occ<P>())) void k_lu_update(Ctx c, int k, int jlo) {
    if (c.dec[k] != 1) return;
    typedef typename Tr<P>::S S;
    if constexpr (P == P32 && NB >= 128) {
        __shared__ __attribute__((aligned(16))) float sm[upd_lds_floats()];
        constexpr int PER = NB / 128;
        const int rest = (int)c.n - k - 1;
        const int b = blockIdx.x, sub = b % (PER * PER), t = b / (PER * PER);
        const int i = k + 1 + t % rest, j = jlo + t / rest;
        const float *At = (const float *)c.At;
        lu_update_f32<NB>(At + c.toff(i, k), At + c.toff(k, j), (float *)c.At + c.toff(i, j), (sub % PER) * 128,
                          (sub / PER) * 128, sm);
        return;
    } else if constexpr (P == P64 && NB >= 128) {
        __shared__ __attribute__((aligned(16))) double sm[upd64_lds_doubles()];
        constexpr int PER = NB / 128;
        const int rest = (int)c.n - k - 1;
        const int b = blockIdx.x, sub = b % (PER * PER), t = b / (PER * PER);
        const int i = k + 1 + t % rest, j = jlo + t / rest;
        const double *At = (const double *)c.At;
        lu_update_f64<NB>(At + c.toff(i, k), At + c.toff(k, j), (double *)c.At + c.toff(i, j), (sub % PER) * 128,
                          (sub / PER) * 128, sm);
        return;
    } else {
    constexpr int BT = upd_bt<NB>();
    constexpr int BK = (P == PB16) ? 32 : 16;
    constexpr int PER = NB / BT;
    __shared__ __attribute__((aligned(16))) char smem[mma_lds_bytes<P, BT, BT, BK>()];
    const int rest = (int)c.n - k - 1;
    int b = blockIdx.x;
    const int sub = b % (PER * PER);
    const int t = b / (PER * PER);
    const int i = k + 1 + t % rest, j = jlo + t / rest;
    const int r0 = (sub % PER) * BT, c0 = (sub / PER) * BT;
    S *At = (S *)c.At;
    const S *Aik = At + c.toff(i, k);
    const S *Akj = At + c.toff(k, j);
    S *Cij = At + c.toff(i, j);
    const float sa = tile_scale<P>(c, i, k), sb = tile_scale<P>(c, k, j);
    typename Tr<P>::acc acc[BT / 2 / 16][BT / 2 / 16];
    acc_zero<P, BT, BT, 2, 2>(acc);
    wg_mma_split<P, BT, BT, 2, 2, BK>(
        acc, NB, [&](int r, int kk) { return (double)Aik[r0 + r + kk * NB] * sa; },
        [&](int kk, int cc) { return (double)Akj[kk + (c0 + cc) * NB] * sb; }, smem);
    const double inv = 1.0 / ((double)sa * (double)sb);
    acc_foreach<P, BT, BT, 2, 2>(acc, [&](int r, int cc, double v) {
        S *p = Cij + (r0 + r) + (size_t)(c0 + cc) * NB;
        *p = (S)((double)*p - v * inv);
    });
    }
}

}  // namespace lq
