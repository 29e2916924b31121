// Shared device helpers and the workspace layout of the MI355X hybrid LU-QR
// solver.  Everything here targets gfx950 (CDNA4): 64-lane wavefronts,
// 256-thread workgroups (4 waves), MFMA 16x16 tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "luqr.h"

#define LQ_DEV __device__ __forceinline__
#define LQ_HD __host__ __device__ __forceinline__

namespace lq {

constexpr int WG = 256;    // threads per workgroup
constexpr int IB = 16;     // inner block of panel factorizations and compact-WY factors
constexpr int WAVE = 64;
constexpr int KRYLOV_MAX = 30;  // largest GMRES basis of luqr_solve_gmres_ir

enum Prec { P64 = 0, P32 = 1, PB16 = 2 };

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Per-precision traits.  S = storage type of the factors, C = compute type of
// the trailing contractions (operands as MFMA sees them), acc = accumulator.
// MFMA 16x16 layout used everywhere (lane l, accumulator register r):
//   A operand:  row l%16,  k = KPL*(l/16) + e  (e < KPL)
//   B operand:  col l%16,  k = KPL*(l/16) + e
//   D / C:      row drow(l/16, r), col l%16, where drow(g, r) = 4g + r for
//               the FP32-accumulating forms and g + 4r for f64 16x16x4
//               (measured on gfx950 with a lane-layout probe)
// KPL = 1 (f64, f32: k-step of 4) or 8 (bf16: k-step of 32).
// ---------------------------------------------------------------------------
template <int P> struct Tr;
template <> struct Tr<P64> {
    typedef double S; typedef double C; typedef d4 acc; typedef double frag;
    static constexpr int KPL = 1;
    static LQ_DEV int drow(int g, int r) { return g + 4 * r; }
    static LQ_DEV acc mma(frag a, frag b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct Tr<P32> {
    typedef float S; typedef float C; typedef f4 acc; typedef float frag;
    static constexpr int KPL = 1;
    static LQ_DEV int drow(int g, int r) { return 4 * g + r; }
    static LQ_DEV acc mma(frag a, frag b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct Tr<PB16> {
    typedef float S; typedef __bf16 C; typedef f4 acc; typedef bf8 frag;
    static constexpr int KPL = 8;
    static LQ_DEV int drow(int g, int r) { return 4 * g + r; }
    static LQ_DEV acc mma(frag a, frag b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <class A> LQ_DEV A zero_acc() { A z; for (int r = 0; r < 4; ++r) z[r] = 0; return z; }

LQ_DEV int lane_id() { return threadIdx.x & 63; }
// uniform over the wave: readfirstlane lets the compiler keep wave-dependent
// values (offsets, loop bounds) in scalar registers
LQ_DEV int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// ---- lane exchanges and wave reductions (64 lanes) ---------------------------
// Six partner maps whose composition reaches every lane: xor 32 and xor 16
// (ds_bpermute across rows), then within each 16-lane row the DPP forms
// row_mirror (i <-> 15-i), row_half_mirror (i <-> 7-i), quad xor 2, quad
// xor 1.  Stage s flips lane bit 5-s (and only lower bits besides), so a
// butterfly over the six stages sums each lane with all 63 others once.
template <int CTRL> LQ_DEV int dpp_i(int x) { return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false); }
template <int ST> LQ_DEV int xlane(int x) {
    if constexpr (ST == 0) return __shfl_xor(x, 32, 64);
    else if constexpr (ST == 1) return __shfl_xor(x, 16, 64);
    else if constexpr (ST == 2) return dpp_i<0x140>(x);  // row_mirror
    else if constexpr (ST == 3) return dpp_i<0x141>(x);  // row_half_mirror
    else if constexpr (ST == 4) return dpp_i<0x4E>(x);   // quad_perm [2,3,0,1]
    else return dpp_i<0xB1>(x);                          // quad_perm [1,0,3,2]
}
template <int ST> LQ_DEV float xlane(float x) { return __int_as_float(xlane<ST>(__float_as_int(x))); }
template <int ST> LQ_DEV double xlane(double x) {
    const int lo = xlane<ST>(__double2loint(x)), hi = xlane<ST>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
// lane bit that distinguishes a lane from its stage-ST partner
template <int ST> constexpr int xbit() { return 5 - ST; }

// Exchange across lane bit 5 (ST = 0) or bit 4 (ST = 1) without LDS:
// v_permlane32_swap / v_permlane16_swap(a, b) swap the upper half-wave
// (odd 16-lane rows) of a with the lower half-wave (even rows) of b.  With
// a = x and b = y the two results hold, in some order, x of this lane and x
// of its partner for lanes with the bit clear, y of this lane and y of its
// partner for lanes with it set; so their sum (or max) is the xor-exchange
// reduction step, and with x = y = v it is v combined with v of the partner
// (checked on every lane with a layout probe).
template <int ST> LQ_DEV void swap_pair(int a, int b, int &r0, int &r1) {
    static_assert(ST == 0 || ST == 1, "permlane swaps exist for lane bits 5 and 4");
    if constexpr (ST == 0) {
        auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        r0 = (int)r[0]; r1 = (int)r[1];
    } else {
        auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        r0 = (int)r[0]; r1 = (int)r[1];
    }
}
// x of this lane plus x (lanes with bit clear) / y (bit set) of the partner,
// laid out as described above: returns keep + received for every lane.
template <int ST> LQ_DEV float swap_add(float x, float y) {
    int r0, r1;
    swap_pair<ST>(__float_as_int(x), __float_as_int(y), r0, r1);
    return __int_as_float(r0) + __int_as_float(r1);
}
template <int ST> LQ_DEV double swap_add(double x, double y) {
    int l0, l1, h0, h1;
    swap_pair<ST>(__double2loint(x), __double2loint(y), l0, l1);
    swap_pair<ST>(__double2hiint(x), __double2hiint(y), h0, h1);
    return __hiloint2double(h0, l0) + __hiloint2double(h1, l1);
}
template <int ST> LQ_DEV double swap_max(double v) {
    int l0, l1, h0, h1;
    swap_pair<ST>(__double2loint(v), __double2loint(v), l0, l1);
    swap_pair<ST>(__double2hiint(v), __double2hiint(v), h0, h1);
    return fmax(__hiloint2double(h0, l0), __hiloint2double(h1, l1));
}

template <class T> LQ_DEV T wave_sum(T v) {
    v = swap_add<0>(v, v); v = swap_add<1>(v, v); v += xlane<2>(v);
    v += xlane<3>(v); v += xlane<4>(v); v += xlane<5>(v);
    return v;
}
LQ_DEV double wave_max(double v) {
    v = swap_max<0>(v); v = swap_max<1>(v); v = fmax(v, xlane<2>(v));
    v = fmax(v, xlane<3>(v)); v = fmax(v, xlane<4>(v)); v = fmax(v, xlane<5>(v));
    return v;
}
template <int ST> LQ_DEV void argmax_step(double &v, int &idx) {
    const double ov = xlane<ST>(v);
    const int oi = xlane<ST>(idx);
    const bool take = (ov > v) | ((ov == v) & (oi < idx));  // selects, no branches
    v = take ? ov : v;
    idx = take ? oi : idx;
}
// argmax of |value| with the smallest index winning ties; NaN never wins.
LQ_DEV void wave_argmax(double &v, int &idx) {
    argmax_step<0>(v, idx); argmax_step<1>(v, idx); argmax_step<2>(v, idx);
    argmax_step<3>(v, idx); argmax_step<4>(v, idx); argmax_step<5>(v, idx);
}

// Sum a 16-vector across the 64 lanes of a wave: stages 0-3 exchange halves
// of the remaining entries (lane bit 5, 4, 3, 2 choosing the upper half),
// stages 4-5 add the last partners.  On return lane l holds the total of
// entry (l >> 2) & 15.
template <int ST, int H, class S> LQ_DEV void xhalf(S (&v)[16]) {
    if constexpr (ST <= 1) {
#pragma unroll
        for (int i = 0; i < H; ++i) v[i] = swap_add<ST>(v[i], v[i + H]);
    } else {
        const bool up = (lane_id() >> xbit<ST>()) & 1;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            S send = up ? v[i] : v[i + H];
            S keep = up ? v[i + H] : v[i];
            v[i] = keep + xlane<ST>(send);
        }
    }
}
template <class S>
LQ_DEV S xreduce16(S (&v)[16]) {
    xhalf<0, 8>(v);
    xhalf<1, 4>(v);
    xhalf<2, 2>(v);
    xhalf<3, 1>(v);
    S t = v[0] + xlane<4>(v[0]);
    return t + xlane<5>(t);
}

// Order LDS traffic between lanes of one wave (no workgroup barrier).
LQ_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- cross-workgroup flags (agent scope) -----------------------------------
// Producer and consumer workgroups of a kernel run on one device, so every
// fence of the flag protocol is agent-scoped (a system-scope fence would also
// write back or invalidate cache lines for host and peer coherence).
LQ_DEV void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
LQ_DEV void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
// The cache half of an agent-scope acquire: invalidate the vector caches so
// later loads see data published by other workgroups.  For use after a
// barrier that follows another thread's completed flag read; unlike
// fence_acquire it does not first wait for this wave's own outstanding
// stores (which need no ordering against the published data).
LQ_DEV void cache_invalidate() { asm volatile("buffer_inv sc1" ::: "memory"); }
LQ_DEV void flag_publish(int *f, int v) {
    fence_release();  // make prior writes of this thread visible
    __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Spin until *f >= v.  Returns false if the spin bound is exhausted.
LQ_DEV bool flag_wait(const int *f, int v, int *watchdog) {
    long spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1L << 26)) {
            __hip_atomic_store(watchdog, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if (__hip_atomic_load(watchdog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    }
    fence_acquire();
    return true;
}

// ---- conversions -----------------------------------------------------------
template <class T> LQ_DEV T cvt(double x);
template <> LQ_DEV double cvt<double>(double x) { return x; }
template <> LQ_DEV float cvt<float>(double x) { return (float)x; }
template <> LQ_DEV __bf16 cvt<__bf16>(double x) { return (__bf16)(float)x; }

// ---------------------------------------------------------------------------
// Device status word.
// ---------------------------------------------------------------------------
struct DevStatus {
    long long info;      // first zero pivot (1-based global row) in an LU step
    int nonfinite;
    int n_lu;
    int ir_iters;
    int ir_converged;
    double ir_eta;
    int watchdog;
    int pad;
};

// ---------------------------------------------------------------------------
// Workspace layout.  All tiles are nb x nb, column-major, tile-major order:
// tile (i,j) of an n x n tile grid starts at (j*n + i)*nb*nb elements.  The
// matrix is padded to Np = n*nb with an identity block, so every kernel works
// on full tiles (the clean-up case of Sec. 2.4 then costs nothing).
// ---------------------------------------------------------------------------
struct Layout {
    int64_t N, n, nb, Np;
    int prec, nrhs_max;
    int dstride;     // diagonal domain: tiles k, k+dstride, ... of the panel (0: the tile alone)
    int64_t DR;      // rows of the largest stacked domain (nb without a domain)
    int qtree;       // QR elimination tree: group size S (0: the flat tree)
    size_t off_WD, off_dperm, off_Tt;
    int64_t sz_S;  // bytes of a storage element
    size_t off_At, off_Tf, off_gram, off_W, off_Linv, off_Dinv, off_ipiv, off_perm, off_zpiv;
    size_t off_dec, off_s, off_m, off_margin, off_status;
    size_t off_tnorm, off_away, off_lmax, off_invpart, off_flags, off_eflag, off_scale;
    size_t off_Y, off_Z, off_X, off_R, off_D, off_Xd, off_G, off_part, off_apart, off_rnorm, off_anorm, off_conv;
    size_t off_kry, off_kdots;  // GMRES refinement: KRYLOV_MAX + 2 vectors of Np doubles; dot scratch
    size_t total;
    int64_t nparts;  // column chunks of the residual kernel
};

LQ_HD size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(int64_t N, int64_t nb, int prec, int nrhs_max, int dstride = 0, int qtree = 0) {
    Layout L;
    L.N = N; L.nb = nb; L.n = (N + nb - 1) / nb; L.Np = L.n * nb;
    L.prec = prec; L.nrhs_max = nrhs_max < 1 ? 1 : nrhs_max;
    L.dstride = dstride;
    L.qtree = qtree;
    L.DR = (dstride > 0 ? 1 + (L.n - 1) / dstride : 1) * nb;
    L.sz_S = prec == P64 ? 8 : 4;
    const size_t n = L.n, b = nb, t2 = b * b;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    L.off_At = take(n * n * t2 * L.sz_S);
    L.off_Tf = take(n * (n + 1) / 2 * t2 * L.sz_S);
    L.off_Tt = take(qtree > 0 ? n * (n + 1) / 2 * t2 * L.sz_S : 8);  // TT factors of the killed heads
    L.off_gram = take(n * t2 * 8);
    L.off_W = take(n * t2 * 8);
    L.off_Linv = take(n * t2 * 8);
    L.off_Dinv = take(n * t2 * 8);
    L.off_ipiv = take(n * b * 4);
    L.off_perm = take(n * b * 4);
    L.off_zpiv = take(n * 4);
    L.off_dec = take(n * 4);
    L.off_s = take(n * 8);
    L.off_m = take(n * 8);
    L.off_margin = take(n * 8);
    L.off_status = take(sizeof(DevStatus));
    L.off_tnorm = take(n * 8);
    L.off_away = take(n * b * 8);
    L.off_lmax = take(b * 8);
    L.off_invpart = take((b / 16 + 1) * b * 8);
    L.off_flags = take(n * (b / IB) * 4 + 64);
    L.off_eflag = take(n * 4);
    L.off_scale = take(n * n * 4);
    L.off_WD = take(L.DR > (int64_t)b ? (size_t)L.DR * b * 8 : 8);
    L.off_dperm = take(L.DR > (int64_t)b ? n * (size_t)L.DR * 4 : 8);
    const size_t Np = L.Np, r = L.nrhs_max;
    L.off_Y = take(Np * r * 8);
    L.off_Z = take(Np * r * 8);
    L.off_X = take(Np * r * 8);
    L.off_R = take(Np * r * 8);
    L.off_D = take(Np * r * 8);
    L.off_Xd = take(Np * r * 8);
    L.off_G = take(Np * r * 8);
    L.nparts = (Np + 2047) / 2048;
    L.off_part = take(L.nparts * Np * r * 8);
    L.off_apart = take(L.nparts * Np * 8);
    L.off_rnorm = take(r * 4 * 8);
    L.off_anorm = take(8);
    L.off_conv = take(16);
    L.off_kry = take(Np * (KRYLOV_MAX + 2) * 8);
    L.off_kdots = take((KRYLOV_MAX + 2) * (64 + 4) * 8);
    L.total = o;
    return L;
}

// Device pointers into one workspace, passed by value to every kernel.
struct Ctx {
    void *At;        // factor tiles, storage precision
    void *Tf;        // compact-WY T factor of every QR panel tile (i,k), i >= k: nb x nb upper
                     // triangular, column-major, at tqoff(i,k); the diagonal IB-blocks are the
                     // per-block factors the QR step uses, the rest is filled after the step
    double *gram;    // per panel tile of the current QR step: V^T V (nb x nb, upper IB-blocks)
    double *W;       // per step: FP64 copy of A_kk, factored in place (L\U)
    double *Linv;    // per step: L_kk^{-1} (unit lower), or Q_kk^T (variant A2)
    double *Dinv;    // per step: inverse of the upper-triangular diagonal factor (U or R)
    int *ipiv;       // per step: GETRF interchanges (local rows)
    int *perm;       // per step: row permutation, (P A)(r,:) = A(perm[r],:)
    int *zpiv;       // per step: first zero pivot of GETRF on the copy (1-based), 0 if none
    int *dec;        // per step: 1 = LU, 0 = QR
    double *s, *m, *margin;
    DevStatus *st;
    double *tnorm;   // per tile row i of the current panel: ||A_ik||_1
    double *away;    // per tile row i: column maxima |A_ik(:,j)| (MUMPS)
    double *lmax;    // column maxima of A_kk before factoring (MUMPS)
    double *invpart; // partial column sums of |A_kk^{-1}| per 64-row block
    int *flags;      // QR-step pipeline: flag[i*(nb/IB) + b] = k+1 once block b of tile i's reflectors is published
    int *eflag;      // per step k: consumers of tile column k+1 that have written tile (k+1,k+1) in QR step k
    unsigned *tmax;  // per tile: bit pattern of max |a| (BF16 scaling), tile-major index (j*n+i)
    double *WD;      // diagonal domain of the current step: stacked FP64 copy (DR x nb), factored
    int *dperm;      // per step: stacked-row permutation of the domain, (P D)(s,:) = D(dperm[s],:)
    int64_t N, n;
    int nb;
    int dstride, DR;
    int a2;          // LU steps of variant A2 (GEQRT of A_kk first; Linv holds Q_kk^T, perm the identity)
    int qtree;       // QR elimination tree: group size S, 0 = flat (see QrTree)
    void *Tt;        // TT factor of every killed head (i,k) of a tree, laid out as Tf
    // tiles in the diagonal domain of step k, and whether tile row i > k is one of them
    LQ_HD int dcount(int64_t k) const { return 1 + (dstride > 0 ? (int)((n - 1 - k) / dstride) : 0); }
    LQ_HD bool indom(int64_t k, int64_t i) const { return dstride > 0 && i > k && (i - k) % dstride == 0; }
    LQ_HD int64_t toff(int64_t i, int64_t j) const { return (j * n + i) * (int64_t)nb * nb; }
    // T factor of panel tile (i,k), i >= k: panels packed one after another
    LQ_HD int64_t tqoff(int64_t i, int64_t k) const { return (k * n - k * (k - 1) / 2 + (i - k)) * (int64_t)nb * nb; }
    LQ_HD int msize(int64_t k) const { return (int)((k < n - 1) ? nb : N - (n - 1) * (int64_t)nb); }
};

// The elimination tree of QR step k (Sec. 2.2, Alg. 3; the two-level
// reduction of Sec. 2.2 and 4.2): the panel tiles k..n-1 in groups of s
// consecutive tiles (s = S, or all of them for S = 0 or S >= n-k: the flat
// tree), a last group of a single tile joining the group before it.  Within
// a group its first tile (the head) eliminates the others with TS kernels
// (Alg. 4a); the heads are then reduced by a binary tree of TT kernels (Alg.
// 4b): at distance d = 1, 2, 4, .. head g eliminates head g+d for g = 0, 2d,
// 4d, ..  Every head but tile k is eliminated exactly once.
struct QrTree {
    int k, n, s, G;
    LQ_HD QrTree(int64_t n_, int64_t k_, int S) : k((int)k_), n((int)n_) {
        const int m = n - k;
        s = (S <= 0 || S >= m) ? m : S;
        G = (m + s - 1) / s;
        if (G > 1 && m - (G - 1) * s == 1) --G;
    }
    LQ_HD int head(int g) const { return k + g * s; }
    LQ_HD int end(int g) const { return g + 1 < G ? k + (g + 1) * s : n; }
    LQ_HD bool is_head(int i) const { return (i - k) % s == 0 && (i - k) / s < G; }
    LQ_HD int npairs(int d) const { return G > d ? (G - d - 1) / (2 * d) + 1 : 0; }
    LQ_HD static int level(int d) { int l = 1; while (d > 1) { d >>= 1; ++l; } return l; }
};

// Flag value of step k's launches: 16 per step, phase 0 for the groups (and
// the A2 panel's GEQRT), 1 + log2(d) for the TT level at distance d.
LQ_HD int qr_epoch(int k, int phase) { return (k + 1) * 16 + phase; }

inline Ctx make_ctx(const Layout &L, void *base, int a2 = 0) {
    char *b = (char *)base;
    Ctx c;
    c.At = b + L.off_At; c.Tf = b + L.off_Tf; c.gram = (double *)(b + L.off_gram); c.W = (double *)(b + L.off_W);
    c.Linv = (double *)(b + L.off_Linv); c.Dinv = (double *)(b + L.off_Dinv);
    c.ipiv = (int *)(b + L.off_ipiv); c.perm = (int *)(b + L.off_perm); c.zpiv = (int *)(b + L.off_zpiv);
    c.dec = (int *)(b + L.off_dec); c.s = (double *)(b + L.off_s); c.m = (double *)(b + L.off_m);
    c.margin = (double *)(b + L.off_margin); c.st = (DevStatus *)(b + L.off_status);
    c.tnorm = (double *)(b + L.off_tnorm); c.away = (double *)(b + L.off_away);
    c.lmax = (double *)(b + L.off_lmax); c.invpart = (double *)(b + L.off_invpart);
    c.flags = (int *)(b + L.off_flags); c.eflag = (int *)(b + L.off_eflag); c.tmax = (unsigned *)(b + L.off_scale);
    c.WD = (double *)(b + L.off_WD); c.dperm = (int *)(b + L.off_dperm);
    c.N = L.N; c.n = L.n; c.nb = (int)L.nb;
    c.dstride = L.dstride; c.DR = (int)L.DR;
    c.a2 = a2;
    c.qtree = L.qtree;
    c.Tt = b + L.off_Tt;
    return c;
}

}  // namespace lq
