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
#include "mma.h"

namespace lq {

// NaN-propagating maximum (a NaN input makes the criterion fail, as in LAPACK's
// treatment of non-finite norms).
LQ_DEV double nmax(double a, double b) { return (b > a || b != b) ? b : a; }
LQ_DEV double wave_nmax(double v) {
    for (int o = 32; o > 0; o >>= 1) v = nmax(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// GETRF of the diagonal tile on its FP64 copy W_k, one workgroup.
// Blocked right-looking: each 32-column panel is staged in LDS and factored
// by wave 0 with wave-level argmax (first index of the largest magnitude wins
// ties); then all four waves apply the interchanges to the other columns,
// solve U12 = L11^{-1} A12 and update A22 -= L21 U12.
// ---------------------------------------------------------------------------
template <int NB, class S>
LQ_DEV void getrf_diag(const Ctx &c, int k) {
    __shared__ double P[32 * NB];   // panel column j at P[j*NB + r] (rows >= p0 used)
    __shared__ double Us[32 * 33];  // 32 x 32 chunk of U12
    __shared__ int piv[32];
    __shared__ int zp;
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    double *W = c.W + (size_t)k * NB * NB;
    const S *A = (const S *)c.At + c.toff(k, k);
    for (int e = tid; e < NB * NB; e += WG) W[e] = (double)A[e];
    for (int col = w; col < NB; col += 4) {
        double v = 0.0;
        for (int r = l; r < NB; r += 64) v = nmax(v, fabs((double)A[r + col * NB]));
        v = wave_nmax(v);
        if (l == 0) c.lmax[col] = v;
    }
    if (tid == 0) zp = 0;
    __syncthreads();
    for (int p0 = 0; p0 < NB; p0 += 32) {
        const int H = NB - p0;
        for (int e = tid; e < H * 32; e += WG) {
            int r = p0 + e % H, j = e / H;
            P[j * NB + r] = W[r + (p0 + j) * NB];
        }
        __syncthreads();
        if (w == 0) {
            for (int cc = 0; cc < 32; ++cc) {
                const int col = p0 + cc;
                double v = -1.0;
                int idx = 0x7fffffff;
                for (int r = col + l; r < NB; r += 64) {
                    double a = fabs(P[cc * NB + r]);
                    if (a > v) { v = a; idx = r; }
                }
                wave_argmax(v, idx);
                if (!(v > 0.0)) {  // exactly zero (or non-numeric) column: no elimination
                    if (l == 0) { piv[cc] = col; if (zp == 0) zp = col + 1; }
                    wave_sync();
                    continue;
                }
                if (l == 0) piv[cc] = idx;
                if (idx != col && l < 32) {
                    double t = P[l * NB + col];
                    P[l * NB + col] = P[l * NB + idx];
                    P[l * NB + idx] = t;
                }
                wave_sync();
                const double pv = P[cc * NB + col];
                for (int r = col + 1 + l; r < NB; r += 64) P[cc * NB + r] /= pv;
                wave_sync();
                for (int j = cc + 1; j < 32; ++j) {
                    const double u = P[j * NB + col];
                    for (int r = col + 1 + l; r < NB; r += 64) P[j * NB + r] -= P[cc * NB + r] * u;
                }
                wave_sync();
            }
        }
        __syncthreads();
        for (int e = tid; e < H * 32; e += WG) {
            int r = p0 + e % H, j = e / H;
            W[r + (p0 + j) * NB] = P[j * NB + r];
        }
        if (tid < 32) c.ipiv[(size_t)k * NB + p0 + tid] = piv[tid];
        for (int col = tid; col < NB; col += WG) {
            if (col >= p0 && col < p0 + 32) continue;
            for (int cc = 0; cc < 32; ++cc) {
                const int r = p0 + cc, pr = piv[cc];
                if (pr != r) {
                    double t = W[r + col * NB];
                    W[r + col * NB] = W[pr + col * NB];
                    W[pr + col * NB] = t;
                }
            }
        }
        __syncthreads();
        if (p0 + 32 < NB) {
            for (int col = p0 + 32 + tid; col < NB; col += WG) {  // U12 = L11^{-1} A12
                double x[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) x[q] = W[p0 + q + col * NB];
#pragma unroll
                for (int q = 0; q < 32; ++q)
#pragma unroll
                    for (int r = q + 1; r < 32; ++r) x[r] -= P[q * NB + p0 + r] * x[q];
#pragma unroll
                for (int q = 0; q < 32; ++q) W[p0 + q + col * NB] = x[q];
            }
            __syncthreads();
            for (int c0 = p0 + 32; c0 < NB; c0 += 32) {  // A22 -= L21 U12, 32 columns at a time
                for (int e = tid; e < 32 * 32; e += WG) {
                    int q = e % 32, j = e / 32;
                    Us[j * 33 + q] = W[p0 + q + (c0 + j) * NB];
                }
                __syncthreads();
                for (int r = p0 + 32 + tid; r < NB; r += WG) {
                    double lr[32];
#pragma unroll
                    for (int q = 0; q < 32; ++q) lr[q] = P[q * NB + r];
                    for (int j = 0; j < 32; ++j) {
                        double s = W[r + (c0 + j) * NB];
#pragma unroll
                        for (int q = 0; q < 32; ++q) s -= lr[q] * Us[j * 33 + q];
                        W[r + (c0 + j) * NB] = s;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (tid == 0) {
        int *pm = c.perm + (size_t)k * NB;
        const int *ip = c.ipiv + (size_t)k * NB;
        for (int r = 0; r < NB; ++r) pm[r] = r;
        for (int cc = 0; cc < NB; ++cc) {
            int p = ip[cc];
            int t = pm[cc]; pm[cc] = pm[p]; pm[p] = t;
        }
        c.zpiv[k] = zp;
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
    if (blockIdx.x == 0) getrf_diag<NB, S>(c, k);
    else tile_norms<NB, S>(c, k, k + (int)blockIdx.x);
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
    int mumps_reading;
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
        const double *W = c.W + (size_t)k * NB * NB;
        double prod_all = 1.0;
        for (int j = 0; j < mk; ++j) prod_all *= fabs(W[j + j * NB]) / c.lmax[j];
        double prod = 1.0, smin = INFINITY, emax = 0.0;
        lu = 1; margin = INFINITY;
        for (int j = 0; j < mk; ++j) {
            const double pj = fabs(W[j + j * NB]);
            const double gf = pj / c.lmax[j];
            double est = a.mumps_reading == 1 ? awayj[j] * gf : a.mumps_reading == 2 ? awayj[j] * prod_all : awayj[j] * prod;
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
