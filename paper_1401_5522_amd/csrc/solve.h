// Solve with the stored factors (Sec. 2.4, second pass): replay the step
// transformations on the right-hand sides in step order, then block
// back-substitution with the upper-triangular factor.  Right-hand sides live
// in FP64 Np x nrhs arrays (leading dimension Np, padded rows zero); factors
// are read in their storage precision and the arithmetic is FP64.
// Every kernel takes an optional device gate: when *gate != 0 (the
// refinement has converged) it returns at once, so a whole refinement loop
// can be enqueued without the host waiting on it.
#pragma once
#include "common.h"

namespace lq {

// Right-hand sides per workgroup (grid.y chunks of this many columns).
template <int NB> constexpr int rq() { return NB >= 512 ? 8 : 16; }

struct SolveArgs {
    double *Y;        // working right-hand sides (Np x nrhs)
    double *Z;        // forward results z_k
    double *X;        // solution
    double *G;        // QR-step scratch (Np x nrhs): Y_ik^T y_i, then the block products W_i
    int nrhs;
    const int *gate;  // may be null
};

LQ_DEV bool gated(const int *g) { return g && *(volatile const int *)g; }

// B (N x nrhs, ldb) -> Y (Np x nrhs), zero padding.
static __global__ void k_rhs_in(const double *B, int64_t ldb, double *Y, int64_t N, int64_t Np, int nrhs, const int *gate) {
    if (gated(gate)) return;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Np * nrhs) return;
    int64_t r = t % Np, q = t / Np;
    Y[t] = r < N ? B[r + q * ldb] : 0.0;
}

static __global__ void k_rhs_out(const double *X, double *B, int64_t ldb, int64_t N, int64_t Np, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t r = t % N, q = t / N;
    B[r + q * ldb] = X[r + q * Np];
}

// ---------------------------------------------------------------------------
// Tile times right-hand-side block, by rows: for the RB = min(64, nb) rows
// [r0, r0+RB) of an nb x nb column-major tile M,
//   acc(r, q) = sum_c M(r, c) v[q*NB + c]   (v in LDS),
// restricted by MODE: 0 every c; 1 c >= r (upper triangle);
// 2 c < r plus a unit diagonal (unit-lower triangle).  The four waves split
// the columns in quarters; each lane owns one row, loads 16 columns of it
// (coalesced across lanes) before using them, and the quarters are summed
// through LDS.  Result for lane l of wave 0: row r0 + l.
// ---------------------------------------------------------------------------
template <int NB> constexpr int mv_rb() { return NB < 64 ? NB : 64; }

template <int NB, int MODE, class S, int RQ>
LQ_DEV bool rows_mv(const S *M, const double *v, int nq, int r0, double (&out)[RQ], double *red) {
    constexpr int QC = NB / 4, U = QC < 16 ? QC : 16;
    const int l = lane_id(), w = wave_id();
    const int r = r0 + l;
    const bool live = l < mv_rb<NB>();
    double acc[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) acc[q] = 0.0;
    if (live) {
        const S *p = M + r;
        for (int c0 = w * QC; c0 < (w + 1) * QC; c0 += U) {
            S a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = p[(size_t)(c0 + u) * NB];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cc = c0 + u;
                double x = (double)a[u];
                if constexpr (MODE == 1) x = cc >= r ? x : 0.0;
                if constexpr (MODE == 2) x = cc < r ? x : (cc == r ? 1.0 : 0.0);
#pragma unroll
                for (int q = 0; q < RQ; ++q)
                    if (q < nq) acc[q] += x * v[q * NB + cc];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (q < nq) red[(w * RQ + q) * 64 + l] = acc[q];
    __syncthreads();
    if (w != 0 || !live) return false;
#pragma unroll
    for (int q = 0; q < RQ; ++q)
        if (q < nq) out[q] = red[q * 64 + l] + red[(RQ + q) * 64 + l] + red[(2 * RQ + q) * 64 + l] +
                             red[(3 * RQ + q) * 64 + l];
    return true;
}

// LU step with a diagonal domain, part 0: the stacked permutation of the
// domain's GEPP on the rows of y in its tiles.  grid (1, rhs chunks of 16).
template <int NB>
static __global__ __launch_bounds__(WG) void k_fwd_dswap(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 1 || gated(s.gate)) return;
    const int d = c.dcount(k);
    if (d < 2) return;
    constexpr int QC = 16;
    __shared__ double buf[512 * QC];
    const int R = d * NB, q0 = blockIdx.y * QC, nq = min(QC, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const int *pm = c.dperm + (size_t)k * c.DR;
    auto row = [&](int sr) { return (k + (int64_t)(sr / NB) * c.dstride) * NB + sr % NB; };
    for (int e = threadIdx.x; e < R * nq; e += WG) buf[e] = s.Y[row(e % R) + (q0 + e / R) * Np];
    __syncthreads();
    for (int e = threadIdx.x; e < R * nq; e += WG) {
        const int r = e % R, sr = pm[r];
        if (sr != r) s.Y[row(r) + (q0 + e / R) * Np] = buf[sr + (e / R) * R];
    }
}

// LU step, part 1: z_k = L^{-1} P y_k (L^{-1} from the panel, FP64; for
// variant A2, z_k = Q_kk^T y_k).
// grid (nb / RB row blocks, rhs chunks).
template <int NB>
static __global__ __launch_bounds__(WG) void k_fwd_lu_a(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 1 || gated(s.gate)) return;
    constexpr int RQ = rq<NB>();
    __shared__ double ys[NB * RQ];
    __shared__ double red[4 * RQ * 64];
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int r0 = blockIdx.x * mv_rb<NB>();
    const int64_t Np = c.n * NB;
    const int *pm = c.perm + (size_t)k * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) {
        const int r = e % NB, q = e / NB;
        ys[q * NB + r] = s.Y[k * NB + pm[r] + (q0 + q) * Np];
    }
    __syncthreads();
    double out[RQ];
    const double *Li = c.Linv + (size_t)k * NB * NB;
    // variant A2: Linv holds the dense Q_kk^T and perm is the identity
    if (c.a2 ? rows_mv<NB, 0>(Li, ys, nq, r0, out, red) : rows_mv<NB, 2>(Li, ys, nq, r0, out, red))
        for (int q = 0; q < nq; ++q) s.Z[k * NB + r0 + lane_id() + (q0 + q) * Np] = out[q];
}

// y_i -= M_i v for the tiles M_i of one tile column (LU: L_ik z_k; QR: Y_ik
// w_i) or tile row (back-substitution: U_ik x_k).  grid (tiles * nb / RB,
// rhs chunks); tile t = blockIdx.x / (nb / RB) is tile row i = i0 + t.
// Source vector: z_k (kind 0), w_i from the QR scratch (kind 1), x_k (kind 2).
template <int NB, class S, int KIND>
LQ_DEV void tile_update(const Ctx &c, const SolveArgs &s, int k, int i0, double *dst) {
    constexpr int RQ = rq<NB>(), RPT = NB / mv_rb<NB>();
    __shared__ double vs[NB * RQ];
    __shared__ double red[4 * RQ * 64];
    const int i = i0 + (int)blockIdx.x / RPT;
    const int r0 = ((int)blockIdx.x % RPT) * mv_rb<NB>();
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const double *src = KIND == 0 ? s.Z + (int64_t)k * NB : KIND == 1 ? s.G + (int64_t)i * NB : s.X + (int64_t)k * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) vs[e] = src[e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    const S *M = (const S *)c.At + c.toff(i, k);
    double out[RQ];
    if (rows_mv<NB, 0>(M, vs, nq, r0, out, red))
        for (int q = 0; q < nq; ++q) dst[(int64_t)i * NB + r0 + lane_id() + (q0 + q) * Np] -= out[q];
}

// LU step, part 2: y_i -= L_ik z_k for i > k.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_lu_b(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 1 || gated(s.gate)) return;
    tile_update<NB, S, 0>(c, s, k, k + 1, s.Y);
}

// out[q*ldo + r] = sum_c M(c, r) u[q*NB + c] for r in [rlo, rhi), q < nq: the
// products M^T u with M an nb x nb column-major tile, where by MODE
//   0: M as stored;  1: upper triangle of M (c <= r);
//   2: unit-lower trapezoid (c > r: stored value, c == r: 1, c < r: 0).
// Each wave takes groups of 16 columns; lanes run down the rows (coalesced
// loads, all issued before use, masks applied by select), keep 16 partial
// sums and combine them with one transpose-reduction.
template <int NB, int NW, int MODE, class S>
LQ_DEV void cols_dot(const S *M, const double *u, int nq, double *out, int64_t ldo, int rlo, int rhi) {
    const int l = lane_id(), w = (int)(threadIdx.x >> 6);
    for (int g = rlo / 16 + w; g < rhi / 16; g += NW) {
        const int r0 = 16 * g;
        const int mlo = MODE == 2 ? r0 / 64 : 0;
        const int mhi = MODE == 1 ? (r0 + 15) / 64 : (NB - 1) / 64;
        for (int q = 0; q < nq; ++q) {
            double v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = 0.0;
            for (int m = mlo; m <= mhi; ++m) {
                const int cc = 64 * m + l;
                if (NB < 64 && cc >= NB) break;  // nb = 32: the upper half-wave idles
                const double uc = u[q * NB + cc];
                S a[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) a[j] = M[cc + (size_t)(r0 + j) * NB];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int r = r0 + j;
                    double x = (double)a[j];
                    if constexpr (MODE == 1) x = cc <= r ? x : 0.0;
                    if constexpr (MODE == 2) x = cc > r ? x : (cc == r ? 1.0 : 0.0);
                    v[j] += x * uc;
                }
            }
            const double tot = xreduce16(v);
            if ((l & 3) == 0) out[q * ldo + r0 + ((l >> 2) & 15)] = tot;
        }
    }
}

// QR step, part 1: g_i = Y_ik^T y_i for i > k.  grid (tiles * QS, rhs
// chunks): QS workgroups share the nb columns of one tile.
template <int NB> constexpr int qs() { return NB >= 128 ? 4 : 1; }

template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_qr_g(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 0 || gated(s.gate)) return;
    constexpr int RQ = rq<NB>(), QS = qs<NB>();
    __shared__ double ys[NB * RQ];
    const int i = k + 1 + (int)blockIdx.x / QS;
    if (QrTree(c.n, k, c.qtree).is_head(i)) return;  // a head's row: its GEQRT in the chain, TT below
    const int part = (int)blockIdx.x % QS;
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) ys[e] = s.Y[i * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    cols_dot<NB, WG / 64, 0, S>((const S *)c.At + c.toff(i, k), ys, nq, s.G + i * NB + q0 * Np, Np,
                                part * (NB / QS), (part + 1) * (NB / QS));
}

// QR step, part 2 (one workgroup per group of the elimination tree and rhs
// chunk; the flat tree is one group headed by tile k): the group's chain
// applied to its head row h.  First z = Q_hh^T y_h = z - V T^T V^T z (GEQRT
// tile), then for the group's tiles i = h+1.. in order, with the full TS
// factor of tile (i,k),
//   w_i = T_ik^T (z + g_i),  z -= w_i,
// which is the top half of [z; y_i] <- Q_ik^T [z; y_i] (V = [I; Y_ik]); the
// bottom half y_i -= Y_ik w_i is independent of the chain and left to part 3.
// Only the triangular T factors are read inside the chain.  z goes to Z_k
// (flat tree) or back to y_h for the TT levels (k_fwd_tt).
// threads of the chain workgroup: eight waves for 4-byte storage (T read into
// registers for n_b <= 256), sixteen for 8-byte storage (T read from memory:
// its registers would not fit beside the rest)
template <int NB, class S> constexpr int chain_wg() { return sizeof(S) == 4 ? 512 : 1024; }

// Buffer loads of a tile: one register holds the lane's offset and each
// load adds a wave-uniform offset from a scalar register, so a run of loads
// in flight costs no address registers per load (with 64-bit addresses it
// cost two each).  Dword 3 is the CDNA raw-buffer format word (32-bit data);
// offsets past the tile read as zero.
LQ_DEV __amdgpu_buffer_rsrc_t tile_rsrc(const float *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, bytes, 0x00020000);
}
LQ_DEV f4 tile_load4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// 16-byte register vector of the storage type
template <class S> struct V16t;
template <> struct V16t<float> { typedef f4 T; };
template <class S> using V16 = typename V16t<S>::T;

// w = T^T u for the upper-triangular T of one panel tile (4-byte storage,
// n_b <= 256), with
// T's entries held in registers, loaded one or two steps of the chain ahead,
// so the chain waits on no global load.  The n_b/16 groups of sixteen output
// columns are dealt to the eight waves: group w and, for n_b = 256, group
// 15 - w (group g needs rows 0 .. 16 g + 15, so the pair balances the
// triangle).  Lane l holds, for output column q = 16 g + 8 h + (l >> 3)
// (h = 0, 1), the rows p = CH m + VE (l & 7) .. + VE - 1 of chunk m: each
// load reads VE consecutive entries (16 bytes) of a column, and one load
// instruction covers eight columns with whole 128-byte lines.  The eight
// lanes of a column are summed with three lane exchanges.
template <int NB, class S> struct ChainR {
    static constexpr int VE = 16 / (int)sizeof(S);  // entries per 16-byte load
    static constexpr int CH = 8 * VE;               // rows per chunk
    static constexpr int NG = NB / 16;
    static constexpr bool PAIR = NG > 8;
    static_assert(NB % CH == 0 && NG <= 16, "register chain: n_b <= 256, chunks divide n_b");
    LQ_DEV static constexpr int nch(int g) { return (16 * g + 16 + CH - 1) / CH; }
    LQ_DEV static constexpr int n0of(int w) { return w < NG ? nch(w) : 0; }
    LQ_DEV static constexpr int ntof(int w) { return n0of(w) + (PAIR ? nch(NG - 1 - w) : 0); }
    static constexpr int maxn() {
        int m = 0;
        for (int w = 0; w < 8; ++w) m = ntof(w) > m ? ntof(w) : m;
        return m;
    }
    static constexpr int NCH = maxn();
    V16<S> t[NCH][2];
    LQ_DEV void load(const S *T) {
        const int w = wave_id(), l = lane_id(), n0 = n0of(w), nt = ntof(w);
        const __amdgpu_buffer_rsrc_t r = tile_rsrc(T, NB * NB * (int)sizeof(S));
        const int voff = (VE * (l & 7) + (l >> 3) * NB) * (int)sizeof(S);
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int g = j < n0 ? w : NG - 1 - w, m = j < n0 ? j : j - n0;
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (j < nt) t[j][h] = tile_load4(r, voff, (CH * m + (16 * g + 8 * h) * NB) * (int)sizeof(S));
        }
    }
    LQ_DEV void apply(const double *u, int nq, double *out) {
        const int w = wave_id(), l = lane_id(), n0 = n0of(w), nt = ntof(w);
        for (int qq = 0; qq < nq; ++qq) {
            // keeps the conversions to FP64 inside the loop over right-hand
            // sides: hoisted out of it they would double the registers of T
#pragma unroll
            for (int j = 0; j < NCH; ++j)
#pragma unroll
                for (int h = 0; h < 2; ++h) asm volatile("" : "+v"(t[j][h]));
            double a[2][2] = {{0.0, 0.0}, {0.0, 0.0}};  // [group slot][h]
#pragma unroll
            for (int j = 0; j < NCH; ++j) {
                if (j >= nt) continue;  // uniform over the wave
                const int g = j < n0 ? w : NG - 1 - w, m = j < n0 ? j : j - n0;
                const int p0 = CH * m + VE * (l & 7);
                double uv[VE];
#pragma unroll
                for (int e = 0; e < VE; ++e) uv[e] = u[qq * NB + p0 + e];
                const bool diag = j == n0 - 1 || j == nt - 1;  // the chunk that reaches the diagonal
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int q = 16 * g + 8 * h + (l >> 3);
                    double d = 0.0;
#pragma unroll
                    for (int e = 0; e < VE; ++e) {
                        double x = (double)t[j][h][e];
                        if (diag) x = p0 + e <= q ? x : 0.0;  // T's strictly lower part is not held
                        d += x * uv[e];
                    }
                    if (j < n0) a[0][h] += d;
                    else a[1][h] += d;
                }
            }
#pragma unroll
            for (int sl = 0; sl < 2; ++sl)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double v = a[sl][h];
                    v += xlane<5>(v);
                    v += xlane<4>(v);
                    v += xlane<3>(v);
                    const bool has = sl == 0 ? n0 > 0 : PAIR;
                    const int g = sl == 0 ? w : NG - 1 - w;
                    if (has && (l & 7) == 0) out[qq * NB + 16 * g + 8 * h + (l >> 3)] = v;
                }
        }
    }
};

template <int NB, class S>
static __global__ __launch_bounds__((chain_wg<NB, S>())) void k_fwd_qr_chain(Ctx c, SolveArgs s, int k) {
    constexpr int CHAIN_WG = chain_wg<NB, S>();
    if (c.dec[k] != 0 || gated(s.gate)) return;
    constexpr int RQ = rq<NB>(), NW = CHAIN_WG / 64;
    constexpr int PER = (NB * RQ + CHAIN_WG - 1) / CHAIN_WG;
    __shared__ double x[NB * RQ], u[NB * RQ], w[NB * RQ];
    const int tid = threadIdx.x;
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const S *At = (const S *)c.At, *Tf = (const S *)c.Tf;
    const QrTree tr(c.n, k, c.qtree);
    const int h = tr.head((int)blockIdx.x), iend = tr.end((int)blockIdx.x);
    const S *V = At + c.toff(h, k);
    auto gidx = [&](int i, int e) { return (int64_t)i * NB + e % NB + (int64_t)(q0 + e / NB) * Np; };
    for (int e = tid; e < NB * nq; e += CHAIN_WG) x[e] = s.Y[gidx(h, e)];
    __syncthreads();
    cols_dot<NB, NW, 2, S>(V, x, nq, u, NB, 0, NB);  // u = V^T z
    __syncthreads();
    cols_dot<NB, NW, 1, S>(Tf + c.tqoff(h, k), u, nq, w, NB, 0, NB);  // w = T^T u
    __syncthreads();
    for (int e = tid; e < NB * nq; e += CHAIN_WG) {  // z -= V w (V unit lower triangular)
        const int r = e % NB, q = e / NB;
        const int rmax = min(NB - 1, r | 63);  // the wave's last row: the loop bound is uniform
        double acc = w[q * NB + r];
        for (int c0 = 0; c0 < rmax; c0 += 32) {  // 32 loads in flight, then the sums in order
            S v[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = V[r + (size_t)(c0 + j) * NB];
#pragma unroll
            for (int j = 0; j < 32; ++j) acc += (c0 + j < r ? (double)v[j] : 0.0) * w[q * NB + c0 + j];
        }
        x[e] -= acc;
    }
    double gn[PER];  // g_i of the next tile row, loaded one iteration ahead
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = tid + p * CHAIN_WG;
        gn[p] = (h + 1 < iend && e < NB * nq) ? s.G[gidx(h + 1, e)] : 0.0;
    }
    // T of the next two tiles in registers (4-byte storage, n_b <= 256)
    constexpr bool REG = NB <= 256 && sizeof(S) == 4;
    constexpr int PD = REG ? 2 : 1;
    ChainR<(REG ? NB : 32), float> ta, tb;
    if constexpr (REG) {
        if (h + 1 < iend) ta.load((const float *)Tf + c.tqoff(h + 1, k));
        if constexpr (PD == 2)
            if (h + 2 < iend) tb.load((const float *)Tf + c.tqoff(h + 2, k));
    }
    auto step = [&](int i, ChainR<(REG ? NB : 32), float> &tc) __attribute__((always_inline)) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = tid + p * CHAIN_WG;
            if (e < NB * nq) u[e] = x[e] + gn[p];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = tid + p * CHAIN_WG;
            gn[p] = (i + 1 < iend && e < NB * nq) ? s.G[gidx(i + 1, e)] : 0.0;
        }
        if constexpr (REG) {
            tc.apply(u, nq, w);
            if (i + PD < iend) tc.load((const float *)Tf + c.tqoff(i + PD, k));
        } else {
            cols_dot<NB, NW, 1, S>(Tf + c.tqoff(i, k), u, nq, w, NB, 0, NB);
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = tid + p * CHAIN_WG;
            if (e < NB * nq) {
                x[e] -= w[e];
                s.G[gidx(i, e)] = w[e];
            }
        }
    };
    for (int i = h + 1; i < iend; i += PD) {
        step(i, ta);
        if constexpr (PD == 2)
            if (i + 1 < iend) step(i + 1, tb);
    }
    double *out = c.qtree ? s.Y : s.Z;  // a tree: the heads' rows go on to the TT levels
    for (int e = tid; e < NB * nq; e += CHAIN_WG) out[gidx(h, e)] = x[e];
}

// QR step with an elimination tree, the TT level at distance d (grid: pairs,
// rhs chunks): [y_h0; y_h1] <- Q^T [y_h0; y_h1] for the TT reflectors V =
// [I; Y] of the killed head h1 (Y upper triangular in tile (h1,k), T in Tt):
// w = T^T (y_h0 + Y^T y_h1), y_h0 -= w, y_h1 -= Y w.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_tt(Ctx c, SolveArgs s, int k, int d) {
    if (c.dec[k] != 0 || gated(s.gate)) return;
    constexpr int RQ = rq<NB>(), NW = WG / 64;
    __shared__ double y0[NB * RQ], y1[NB * RQ], u[NB * RQ], w[NB * RQ];
    __shared__ double red[4 * RQ * 64];
    const QrTree tr(c.n, k, c.qtree);
    const int g0 = 2 * d * (int)blockIdx.x;
    const int h0 = tr.head(g0), h1 = tr.head(g0 + d);
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    auto gidx = [&](int i, int e) { return (int64_t)i * NB + e % NB + (int64_t)(q0 + e / NB) * Np; };
    const S *Y = (const S *)c.At + c.toff(h1, k);
    const S *T = (const S *)c.Tt + c.tqoff(h1, k);
    for (int e = threadIdx.x; e < NB * nq; e += WG) {
        y0[e] = s.Y[gidx(h0, e)];
        y1[e] = s.Y[gidx(h1, e)];
    }
    __syncthreads();
    cols_dot<NB, NW, 1, S>(Y, y1, nq, u, NB, 0, NB);  // u = Y^T y1 (upper triangle of the tile)
    __syncthreads();
    for (int e = threadIdx.x; e < NB * nq; e += WG) u[e] += y0[e];
    __syncthreads();
    cols_dot<NB, NW, 1, S>(T, u, nq, w, NB, 0, NB);  // w = T^T u
    __syncthreads();
    for (int e = threadIdx.x; e < NB * nq; e += WG) s.Y[gidx(h0, e)] = y0[e] - w[e];
    for (int r0 = 0; r0 < NB; r0 += mv_rb<NB>()) {  // y1 -= Y w
        double out[RQ];
        if (rows_mv<NB, 1>(Y, w, nq, r0, out, red))
            for (int q = 0; q < nq; ++q) s.Y[gidx(h1, r0 + lane_id() + q * NB)] = y1[q * NB + r0 + lane_id()] - out[q];
        __syncthreads();
    }
}

// After the TT levels: z_k = y_k (the eliminator row's transformed right-hand
// sides, for the back substitution).
template <int NB>
static __global__ __launch_bounds__(WG) void k_fwd_tt_fin(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 0 || gated(s.gate)) return;
    const int64_t Np = c.n * NB;
    for (int64_t e = blockIdx.x * (int64_t)WG + threadIdx.x; e < (int64_t)NB * s.nrhs; e += (int64_t)gridDim.x * WG)
        s.Z[(int64_t)k * NB + e % NB + (e / NB) * Np] = s.Y[(int64_t)k * NB + e % NB + (e / NB) * Np];
}

// QR step, part 3: y_i -= Y_ik w_i for i > k.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_qr_u(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 0 || gated(s.gate)) return;
    if (QrTree(c.n, k, c.qtree).is_head(k + 1 + (int)blockIdx.x / (NB / mv_rb<NB>()))) return;
    tile_update<NB, S, 1>(c, s, k, k + 1, s.Y);
}

// ---------------------------------------------------------------------------
// The forward pass as one wavefront launch (n_b = 256, 4-byte storage, no
// diagonal domain).  Workgroup k replays step k on the right-hand sides tile
// row by tile row, each as soon as step k-1 has finished with it, so the
// steps overlap: a QR step's chain is sequential over its tile rows, but the
// chains of different steps are not, and one step at a time left all but one
// compute unit idle.  cnt[i] (one array per right-hand-side chunk) counts
// the steps applied to y_i: workgroup k waits until cnt[i] >= k and sets it
// to k+1 once y_i is updated.  y is written and read with agent-scope
// atomic stores and loads (coherent across the chip's L2 caches), the
// writer waits for its stores to complete before the counter is set, so no
// cache writeback or invalidation is needed for the handoff.  A workgroup
// waits only on lower-numbered ones, which are dispatched first, so the
// launch completes whatever the residency.
// A 256 x 256 column-major FP32 tile in registers over 512 threads: lane l
// of wave w holds rows 4l..4l+3 of columns 32w..32w+31, one 16-byte load per
// column, so a wave reads a whole column per instruction and all 32 loads
// are in flight together.  Arithmetic in FP64, as in the per-step kernels.
// ---------------------------------------------------------------------------
constexpr int FW_WG = 512;
constexpr int FW_RQ = 4;  // right-hand sides per workgroup

struct FwTile {
    f4 v[32];
    LQ_DEV void load(const float *M) {
        const int w = wave_id(), l = lane_id();
        const __amdgpu_buffer_rsrc_t r = tile_rsrc(M, 256 * 256 * 4);
        const int voff = (4 * l + 32 * w * 256) * 4;
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = tile_load4(r, voff + (j & 3) * 1024, (j >> 2) * 4096);  // imm + 8 scalars
    }
    // keeps the conversions to FP64 inside the loop over right-hand sides
    // (hoisted, they would double the registers of the tile)
    LQ_DEV void pin() {
#pragma unroll
        for (int j = 0; j < 32; ++j) asm volatile("" : "+v"(v[j]));
    }
};
// entry (p, c) as used by MODE: 0 as stored; 1 upper triangle (p <= c);
// 2 unit lower (below the diagonal as stored, 1 on it, 0 above)
template <int MODE> LQ_DEV double fw_x(float m, int p, int c) {
    if constexpr (MODE == 0) return (double)m;
    else if constexpr (MODE == 1) return p <= c ? (double)m : 0.0;
    else return p > c ? (double)m : (p == c ? 1.0 : 0.0);
}
// out[q*256 + c] = sum_p M(p, c) v[q*256 + p]   (v and out in LDS)
template <int MODE> LQ_DEV void fw_cols(FwTile &t, const double *v, int nq, double *out) {
    const int w = wave_id(), l = lane_id();
    for (int q = 0; q < nq; ++q) {
        t.pin();
        double vv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) vv[e] = v[q * 256 + 4 * l + e];
#pragma unroll
        for (int hb = 0; hb < 2; ++hb) {  // sixteen columns at a time (registers)
            double s0[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                double a = 0.0;
#pragma unroll
                for (int e = 0; e < 4; ++e) a += fw_x<MODE>(t.v[16 * hb + j][e], 4 * l + e, 32 * w + 16 * hb + j) * vv[e];
                s0[j] = a;
            }
            const double a = xreduce16(s0);
            if ((l & 3) == 0) out[q * 256 + 32 * w + 16 * hb + ((l >> 2) & 15)] = a;
        }
    }
}
// red[(w*nq + q)*256 + p] = sum over wave w's 32 columns of M(p, c) v[q*256 + c]
template <int MODE> LQ_DEV void fw_rows(FwTile &t, const double *v, int nq, double *red) {
    const int w = wave_id(), l = lane_id();
    for (int q = 0; q < nq; ++q) {
        t.pin();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const double vc = v[q * 256 + 32 * w + j];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] += fw_x<MODE>(t.v[j][e], 4 * l + e, 32 * w + j) * vc;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) red[(w * nq + q) * 256 + 4 * l + e] = acc[e];
    }
}
// The same row products for an FP64 256 x 256 matrix, by MODE: 0 as stored
// (variant A2's Q_kk^T); 1 upper triangle (the diagonal factor's inverse of
// the back substitution); 2 unit lower (L_kk^{-1}).  Four passes of 8
// columns per wave: lane l holds rows 2l, 2l+1 and 128+2l, 128+2l+1.
template <int MODE>
LQ_DEV void fw_rows_d(const double *M, const double *v, int nq, double *red) {
    const int w = wave_id(), l = lane_id();
    double acc[FW_RQ][4];
#pragma unroll
    for (int q = 0; q < FW_RQ; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[q][e] = 0.0;
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        d2 a[8][2];
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                a[j][h] = *(const d2 *)(M + 128 * h + 2 * l + (size_t)(32 * w + 8 * pass + j) * 256);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int cc = 32 * w + 8 * pass + j;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int p = 128 * h + 2 * l + e;
                    const double x = MODE == 0 ? a[j][h][e]
                                     : MODE == 1 ? (p <= cc ? a[j][h][e] : 0.0)
                                                 : (p > cc ? a[j][h][e] : (p == cc ? 1.0 : 0.0));
#pragma unroll
                    for (int q = 0; q < FW_RQ; ++q)
                        if (q < nq) acc[q][2 * h + e] += x * v[q * 256 + cc];
                }
        }
    }
#pragma unroll
    for (int q = 0; q < FW_RQ; ++q)
        if (q < nq)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e) red[(w * nq + q) * 256 + 128 * h + 2 * l + e] = acc[q][2 * h + e];
}

template <int NB, class S>
static __global__ __launch_bounds__(FW_WG) void k_fwd_wave(Ctx c, SolveArgs s, int *cnt) {
    static_assert(NB == 256 && sizeof(S) == 4, "wavefront forward pass: n_b = 256, 4-byte storage");
    if (gated(s.gate)) return;
    __shared__ double yi[256 * FW_RQ], z[256 * FW_RQ], u[256 * FW_RQ];
    __shared__ double red[8 * 256 * FW_RQ];
    __shared__ int bail;
    const int k = blockIdx.x, n = (int)c.n, tid = threadIdx.x;
    const int q0 = blockIdx.y * FW_RQ, nq = min(FW_RQ, s.nrhs - q0);
    int *cn = cnt + (size_t)blockIdx.y * n;
    const int64_t Np = (int64_t)n * 256;
    const float *At = (const float *)c.At, *Tf = (const float *)c.Tf;
    auto gy = [&](int i, int e) { return (int64_t)i * 256 + e % 256 + (int64_t)(q0 + e / 256) * Np; };
    auto ld = [&](int64_t idx) { return __hip_atomic_load(s.Y + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    auto wait = [&](int i) __attribute__((always_inline)) {
        if (tid == 0) {
            long spins = 0;
            bail = 0;
            while (__hip_atomic_load(cn + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1L << 27) ||
                    __hip_atomic_load(&c.st->watchdog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(&c.st->watchdog, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bail = 1;
                    break;
                }
            }
        }
        __syncthreads();
        return !bail;
    };
    auto publish = [&](int i) __attribute__((always_inline)) {
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores of y_i have completed
        __syncthreads();
        if (tid == 0) __hip_atomic_store(cn + i, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // y_i -= (sum of the waves' row partials), then y_i is published
    auto update_tile = [&](int i) __attribute__((always_inline)) {
        __syncthreads();
        for (int e = tid; e < 256 * nq; e += FW_WG) {
            const int q = e / 256, p = e % 256;
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < 8; ++w) t += red[(w * nq + q) * 256 + p];
            __hip_atomic_store(s.Y + gy(i, e), yi[e] - t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        publish(i);
    };
    FwTile ty;
    if (c.dec[k] == 1) {  // LU step: z_k = L_kk^{-1} P y_k, then y_i -= L_ik z_k
        if (!wait(k)) return;
        const int *pm = c.perm + (size_t)k * 256;
        for (int e = tid; e < 256 * nq; e += FW_WG) yi[e] = ld((int64_t)k * 256 + pm[e % 256] + (int64_t)(q0 + e / 256) * Np);
        __syncthreads();
        if (c.a2) fw_rows_d<0>(c.Linv + (size_t)k * 256 * 256, yi, nq, red);  // A2: the dense Q_kk^T
        else fw_rows_d<2>(c.Linv + (size_t)k * 256 * 256, yi, nq, red);
        __syncthreads();
        for (int e = tid; e < 256 * nq; e += FW_WG) {
            const int q = e / 256, p = e % 256;
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < 8; ++w) t += red[(w * nq + q) * 256 + p];
            z[e] = t;
            s.Z[gy(k, e)] = t;
        }
        if (k + 1 < n) ty.load(At + c.toff(k + 1, k));
        for (int i = k + 1; i < n; ++i) {
            if (!wait(i)) return;
            for (int e = tid; e < 256 * nq; e += FW_WG) yi[e] = ld(gy(i, e));
            fw_rows<0>(ty, z, nq, red);
            if (i + 1 < n) ty.load(At + c.toff(i + 1, k));
            update_tile(i);
        }
        return;
    }
    // QR step: x = Q_kk^T y_k (GEQRT tile), then for i = k+1.. the flat tree:
    // g = Y_ik^T y_i, w = T_ik^T (x + g), x -= w, y_i -= Y_ik w
    ChainR<256, float> tc;
    ty.load(At + c.toff(k, k));
    if (!wait(k)) return;
    for (int e = tid; e < 256 * nq; e += FW_WG) z[e] = ld(gy(k, e));
    __syncthreads();
    fw_cols<2>(ty, z, nq, u);  // u = V^T x
    tc.load(Tf + c.tqoff(k, k));
    __syncthreads();
    tc.apply(u, nq, yi);       // w = T^T u (yi as scratch)
    ty.load(At + c.toff(k, k));
    __syncthreads();
    fw_rows<2>(ty, yi, nq, red);
    __syncthreads();
    for (int e = tid; e < 256 * nq; e += FW_WG) {
        const int q = e / 256, p = e % 256;
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) t += red[(w * nq + q) * 256 + p];
        z[e] -= t;
    }
    for (int i = k + 1; i < n; ++i) {
        // Y_ik is loaded before the wait, T_ik after it and Y_ik again after
        // w (holding Y_ik through w as well would exceed the registers)
        ty.load(At + c.toff(i, k));
        if (!wait(i)) return;  // (its barrier also orders the update of x above)
        tc.load(Tf + c.tqoff(i, k));
        for (int e = tid; e < 256 * nq; e += FW_WG) yi[e] = ld(gy(i, e));
        __syncthreads();
        fw_cols<0>(ty, yi, nq, u);  // g
        __syncthreads();
        for (int e = tid; e < 256 * nq; e += FW_WG) u[e] += z[e];
        __syncthreads();
        double *wv = red + 7 * 256 * FW_RQ;  // w_i: the last wave's slot of red is free until fw_rows
        tc.apply(u, nq, wv);
        ty.load(At + c.toff(i, k));
        __syncthreads();
        for (int e = tid; e < 256 * nq; e += FW_WG) {
            const double t = wv[e];
            z[e] -= t;
            u[e] = t;
        }
        __syncthreads();
        fw_rows<0>(ty, u, nq, red);
        update_tile(i);
    }
    __syncthreads();
    for (int e = tid; e < 256 * nq; e += FW_WG) s.Z[gy(k, e)] = z[e];
}

// Back-substitution, part 1: x_k = D_k^{-1} z_k (D_k = U or R of step k;
// its FP64 inverse is upper triangular).  grid (nb / RB, rhs chunks).
// ---------------------------------------------------------------------------
// The back substitution as one wavefront launch (n_b = 256, 4-byte storage):
// workgroup b solves tile row k = n-1-b,
//     x_k = D_k^{-1} (z_k - sum_{j>k} U_kj x_j),
// with D_k^{-1} the FP64 inverse of the diagonal factor (U or R) and U_kj the
// stored tiles, taking each x_j (j = n-1 down to k+1) as soon as workgroup
// n-1-j has published it (cnt[j] = 1, one array per right-hand-side chunk),
// so the tile products of different rows overlap and only the chain of the
// last product and the diagonal solve is sequential.  x is written and read
// with agent-scope atomics, as y in the forward pass; a workgroup waits only
// on lower-numbered ones, which are dispatched first.
// ---------------------------------------------------------------------------
template <int NB, class S>
static __global__ __launch_bounds__(FW_WG) void k_bwd_wave(Ctx c, SolveArgs s, int *cnt) {
    static_assert(NB == 256 && sizeof(S) == 4, "wavefront back substitution: n_b = 256, 4-byte storage");
    if (gated(s.gate)) return;
    __shared__ double zk[256 * FW_RQ], xv[256 * FW_RQ];
    __shared__ double red[8 * 256 * FW_RQ];
    __shared__ int bail;
    const int n = (int)c.n, k = n - 1 - (int)blockIdx.x, tid = threadIdx.x;
    const int q0 = blockIdx.y * FW_RQ, nq = min(FW_RQ, s.nrhs - q0);
    int *cn = cnt + (size_t)blockIdx.y * n;
    const int64_t Np = (int64_t)n * 256;
    const float *At = (const float *)c.At;
    auto gx = [&](int i, int e) { return (int64_t)i * 256 + e % 256 + (int64_t)(q0 + e / 256) * Np; };
    auto wait = [&](int j) __attribute__((always_inline)) {
        if (tid == 0) {
            long spins = 0;
            bail = 0;
            while (__hip_atomic_load(cn + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 1) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1L << 27) ||
                    __hip_atomic_load(&c.st->watchdog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(&c.st->watchdog, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bail = 1;
                    break;
                }
            }
        }
        __syncthreads();
        return !bail;
    };
    auto sum_red = [&](int e) __attribute__((always_inline)) {
        const int q = e / 256, p = e % 256;
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) t += red[(w * nq + q) * 256 + p];
        return t;
    };
    for (int e = tid; e < 256 * nq; e += FW_WG) zk[e] = s.Z[gx(k, e)];
    FwTile tu;
    if (k + 1 < n) tu.load(At + c.toff(k, n - 1));
    for (int j = n - 1; j > k; --j) {
        if (!wait(j)) return;
        for (int e = tid; e < 256 * nq; e += FW_WG)
            xv[e] = __hip_atomic_load(s.X + gx(j, e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        fw_rows<0>(tu, xv, nq, red);  // U_kj x_j
        if (j - 1 > k) tu.load(At + c.toff(k, j - 1));
        __syncthreads();
        for (int e = tid; e < 256 * nq; e += FW_WG) zk[e] -= sum_red(e);
        __syncthreads();
    }
    fw_rows_d<1>(c.Dinv + (size_t)k * 256 * 256, zk, nq, red);  // D_k^{-1} (upper triangular)
    __syncthreads();
    for (int e = tid; e < 256 * nq; e += FW_WG)
        __hip_atomic_store(s.X + gx(k, e), sum_red(e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores of x_k have completed
    __syncthreads();
    if (tid == 0) __hip_atomic_store(cn + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NB>
static __global__ __launch_bounds__(WG) void k_bwd_a(Ctx c, SolveArgs s, int k) {
    if (gated(s.gate)) return;
    constexpr int RQ = rq<NB>();
    __shared__ double zs[NB * RQ];
    __shared__ double red[4 * RQ * 64];
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int r0 = blockIdx.x * mv_rb<NB>();
    const int64_t Np = c.n * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) zs[e] = s.Z[k * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    double out[RQ];
    if (rows_mv<NB, 1>(c.Dinv + (size_t)k * NB * NB, zs, nq, r0, out, red))
        for (int q = 0; q < nq; ++q) s.X[k * NB + r0 + lane_id() + (q0 + q) * Np] = out[q];
}

// Back-substitution, part 2: z_i -= U_ik x_k for i < k.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_bwd_b(Ctx c, SolveArgs s, int k) {
    if (gated(s.gate)) return;
    tile_update<NB, S, 2>(c, s, k, 0, s.Z);
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement: r = b - A x from the caller's FP64 A.
// ---------------------------------------------------------------------------
constexpr int RCHUNK = 2048;  // columns per residual partial
constexpr int RQR = 8;        // right-hand sides per residual pass

// part[p][q][row] = sum over columns in chunk p of A(row, c) x(c, q); also
// apart[p][row] = sum |A(row, c)| on the first call (for ||A||_inf).
static __global__ __launch_bounds__(WG) void k_resid_part(const double *A, int64_t lda, int64_t N, int64_t Np,
                                                   const double *X, int nrhs, double *part, double *apart,
                                                   const int *gate) {
    if (gated(gate)) return;
    const int64_t r = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int p = blockIdx.y;
    const int q0 = blockIdx.z * RQR, nq = min(RQR, nrhs - q0);
    const int64_t c0 = (int64_t)p * RCHUNK, c1 = min<int64_t>(N, c0 + RCHUNK);
    if (r >= N) return;
    double acc[RQR];
    for (int q = 0; q < RQR; ++q) acc[q] = 0.0;
    double as = 0.0;
    for (int64_t cc = c0; cc < c1; ++cc) {
        const double a = A[r + cc * lda];
        as += fabs(a);
#pragma unroll
        for (int q = 0; q < RQR; ++q)
            if (q < nq) acc[q] += a * X[cc + (q0 + q) * Np];
    }
    const int64_t nparts = gridDim.y;
    for (int q = 0; q < nq; ++q) part[((int64_t)(q0 + q) * nparts + p) * Np + r] = acc[q];
    if (apart && blockIdx.z == 0) apart[(int64_t)p * Np + r] = as;
}

LQ_DEV void atomic_max_nonneg(double *addr, double v) {
    // IEEE order of non-negative doubles equals the order of their bit patterns
    atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

// r = b - sum_p part; ||r||_inf, ||x||_inf per column; ||A||_inf if apart.
static __global__ __launch_bounds__(WG) void k_resid_final(const double *B, int64_t ldb, int64_t N, int64_t Np, int nrhs,
                                                    int nparts, const double *part, const double *apart,
                                                    const double *X, double *R, double *norms, const int *gate) {
    if (gated(gate)) return;
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= N * nrhs) return;
    const int64_t r = t % N;
    const int q = (int)(t / N);
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[((int64_t)q * nparts + p) * Np + r];
    const double res = B[r + q * ldb] - s;
    R[r + q * Np] = res;
    atomic_max_nonneg(&norms[q], fabs(res));
    atomic_max_nonneg(&norms[nrhs + q], fabs(X[r + q * Np]));
    if (apart && q == 0) {
        double as = 0.0;
        for (int p = 0; p < nparts; ++p) as += apart[(int64_t)p * Np + r];
        atomic_max_nonneg(&norms[2 * nrhs], as);
    }
}

// Convergence test: every column has ||r||_inf <= N 1e-16 ||A||_inf ||x||_inf.
// conv[0] = converged flag (gate of the remaining kernels), norms reset.
static __global__ void k_ir_check(double *norms, int nrhs, int64_t N, int *conv, DevStatus *st, int final_check) {
    if (threadIdx.x != 0) return;
    if (conv[0]) return;
    const double anorm = norms[2 * nrhs];
    double eta = 0.0;
    int ok = 1;
    for (int q = 0; q < nrhs; ++q) {
        const double rn = norms[q], xn = norms[nrhs + q];
        const double e = rn / (anorm * xn);
        eta = (e > eta || e != e) ? e : eta;
        if (!(rn <= (double)N * 1e-16 * anorm * xn)) ok = 0;
    }
    st->ir_eta = eta;
    st->ir_converged = ok;
    if (ok) conv[0] = 1;
    else if (!final_check) st->ir_iters += 1;
    for (int q = 0; q < 2 * nrhs; ++q) norms[q] = 0.0;
}

// x += d (columns of Np rows).
static __global__ void k_ir_update(double *X, const double *D, int64_t total, const int *gate) {
    if (gated(gate)) return;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) X[t] += D[t];
}

// Tile-major factors -> column-major FP64 (N x N, ldf).
template <class S>
static __global__ void k_from_tiles(const S *At, int64_t n, int nb, int64_t N, double *F, int64_t ldf) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    int64_t r = t % N, cc = t / N;
    int64_t i = r / nb, j = cc / nb;
    F[r + cc * ldf] = (double)At[(j * n + i) * (int64_t)nb * nb + (r % nb) + (cc % nb) * (int64_t)nb];
}

// Column-major FP64 A (lda) -> tile-major storage with identity padding.  One
// workgroup per tile (blockIdx.x = i + j n); each lane converts four
// consecutive rows of one column (nb is a multiple of 4), one 4-element store.
template <class S>
static __global__ void k_to_tiles(const double *A, int64_t lda, int64_t N, int64_t n, int nb, S *At) {
    struct alignas(4 * sizeof(S)) S4 { S v[4]; };
    const int64_t tile = blockIdx.x, i = tile % n, j = tile / n;
    S *T = At + tile * (int64_t)nb * nb;
    for (int e = 4 * (int)threadIdx.x; e < nb * nb; e += 4 * (int)blockDim.x) {
        const int64_t r = i * nb + e % nb, cc = j * nb + e / nb;
        S4 o;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            o.v[u] = (S)((r + u < N && cc < N) ? A[r + u + cc * lda] : (r + u == cc ? 1.0 : 0.0));
        *(S4 *)(T + e) = o;
    }
}

static __global__ void k_fill_int(int *p, int64_t count, int v) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}
static __global__ void k_fill_u32(unsigned *p, int64_t count) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = 0u;
}
static __global__ void k_fill_f64(double *p, int64_t count) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = 0.0;
}
static __global__ void k_status_reset(DevStatus *st) {
    if (threadIdx.x == 0) {
        st->info = 0; st->nonfinite = 0; st->n_lu = 0; st->ir_iters = 0; st->ir_converged = 0;
        st->ir_eta = 0.0; st->watchdog = 0; st->pad = 0;
    }
}
static __global__ void k_ir_reset(DevStatus *st, int *conv) {
    if (threadIdx.x == 0) { st->ir_iters = 0; st->ir_converged = 0; st->ir_eta = 0.0; conv[0] = 0; conv[1] = 0; }
}

}  // namespace lq
