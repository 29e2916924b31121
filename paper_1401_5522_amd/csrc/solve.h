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

constexpr int RQ = 16;  // right-hand sides per workgroup

struct SolveArgs {
    double *Y;        // working right-hand sides (Np x nrhs)
    double *Z;        // forward results z_k
    double *X;        // solution
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

// LU step, part 1: z_k = L^{-1} P y_k.  grid.y = rhs chunks.
template <int NB>
static __global__ __launch_bounds__(WG) void k_fwd_lu_a(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 1 || gated(s.gate)) return;
    __shared__ double ys[NB * RQ];
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const int *pm = c.perm + (size_t)k * NB;
    const double *Li = c.Linv + (size_t)k * NB * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) {
        int r = e % NB, q = e / NB;
        ys[q * NB + r] = s.Y[k * NB + pm[r] + (q0 + q) * Np];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NB * nq; e += WG) {
        int r = e % NB, q = e / NB;
        double acc = ys[q * NB + r];
        for (int cc = 0; cc < r; ++cc) acc += Li[r + (size_t)cc * NB] * ys[q * NB + cc];
        s.Z[k * NB + r + (q0 + q) * Np] = acc;
    }
}

// LU step, part 2: y_i -= L_ik z_k for i > k (one workgroup per tile row).
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_lu_b(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 1 || gated(s.gate)) return;
    __shared__ double zs[NB * RQ];
    const int i = k + 1 + blockIdx.x;
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) zs[e] = s.Z[k * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    const S *L = (const S *)c.At + c.toff(i, k);
    for (int r = threadIdx.x; r < NB; r += WG) {
        double acc[RQ];
        for (int q = 0; q < RQ; ++q) acc[q] = 0.0;
        for (int cc = 0; cc < NB; ++cc) {
            double a = (double)L[r + cc * NB];
#pragma unroll
            for (int q = 0; q < RQ; ++q)
                if (q < nq) acc[q] += a * zs[q * NB + cc];
        }
#pragma unroll
        for (int q = 0; q < RQ; ++q)
            if (q < nq) s.Y[i * NB + r + (q0 + q) * Np] -= acc[q];
    }
}

// Apply one compact-WY block (IB reflectors starting at row c0 of the
// eliminator) to right-hand-side blocks held in LDS.  TS form (Yb given):
// W = T^T (zk[c0..c0+IB) + Y^T yi); zk[c0..] -= W; yi -= Y W.
// GEQRT form (Yb null, V = unit-lower columns of the diagonal tile):
// W = T^T V^T zk; zk -= V W.
template <int NB, class S>
LQ_DEV void fwd_block(double *zk, double *yi, const S *Vt, const S *Yb, const S *Tt, int c0, int nq, double *Wsh) {
    const int tid = threadIdx.x;
    for (int e = tid; e < IB * nq; e += WG) {
        int lq = e % IB, q = e / IB;
        double acc;
        if (Yb) {
            acc = zk[q * NB + c0 + lq];
            for (int r = 0; r < NB; ++r) acc += (double)Yb[r + (c0 + lq) * NB] * yi[q * NB + r];
        } else {
            acc = zk[q * NB + c0 + lq];
            for (int r = c0 + lq + 1; r < NB; ++r) acc += (double)Vt[r + (c0 + lq) * NB] * zk[q * NB + r];
        }
        Wsh[q * IB + lq] = acc;
    }
    __syncthreads();
    double w2[(IB * RQ + WG - 1) / WG];
    int u = 0;
    for (int e = tid; e < IB * nq; e += WG, ++u) {
        int lq = e % IB, q = e / IB;
        double acc = 0.0;
        for (int p = 0; p <= lq; ++p) acc += (double)Tt[(c0 + p) + lq * NB] * Wsh[q * IB + p];
        w2[u] = acc;
    }
    __syncthreads();
    u = 0;
    for (int e = tid; e < IB * nq; e += WG, ++u) Wsh[(e / IB) * IB + e % IB] = w2[u];
    __syncthreads();
    if (Yb) {
        for (int e = tid; e < IB * nq; e += WG) zk[(e / IB) * NB + c0 + e % IB] -= Wsh[e];
        for (int e = tid; e < NB * nq; e += WG) {
            int r = e % NB, q = e / NB;
            double acc = 0.0;
            for (int lq = 0; lq < IB; ++lq) acc += (double)Yb[r + (c0 + lq) * NB] * Wsh[q * IB + lq];
            yi[q * NB + r] -= acc;
        }
    } else {
        for (int e = tid; e < (NB - c0) * nq; e += WG) {
            int r = c0 + e % (NB - c0), q = e / (NB - c0);
            double acc = 0.0;
            const int lm = r - c0 < IB ? r - c0 : IB - 1;
            for (int lq = 0; lq <= lm; ++lq) {
                double v = (r == c0 + lq) ? 1.0 : (double)Vt[r + (c0 + lq) * NB];
                acc += v * Wsh[q * IB + lq];
            }
            zk[q * NB + r] -= acc;
        }
    }
    __syncthreads();
}

// QR step: z_k = Q^T-chain applied to (y_k, y_{k+1}, ..., y_{n-1}); one
// workgroup per rhs chunk walks the flat tree in order.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_fwd_qr(Ctx c, SolveArgs s, int k) {
    if (c.dec[k] != 0 || gated(s.gate)) return;
    __shared__ double zk[NB * RQ];
    __shared__ double yi[NB * RQ];
    __shared__ double Wsh[IB * RQ];
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const S *At = (const S *)c.At;
    const S *Tf = (const S *)c.Tf;
    for (int e = threadIdx.x; e < NB * nq; e += WG) zk[e] = s.Y[k * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    const S *Tkk = Tf + c.toff(k, k) / NB * IB;
    for (int c0 = 0; c0 < NB; c0 += IB) fwd_block<NB, S>(zk, yi, At + c.toff(k, k), nullptr, Tkk, c0, nq, Wsh);
    for (int i = k + 1; i < c.n; ++i) {
        for (int e = threadIdx.x; e < NB * nq; e += WG) yi[e] = s.Y[i * NB + e % NB + (q0 + e / NB) * Np];
        __syncthreads();
        const S *Y = At + c.toff(i, k);
        const S *T = Tf + c.toff(i, k) / NB * IB;
        for (int c0 = 0; c0 < NB; c0 += IB) fwd_block<NB, S>(zk, yi, nullptr, Y, T, c0, nq, Wsh);
        for (int e = threadIdx.x; e < NB * nq; e += WG) s.Y[i * NB + e % NB + (q0 + e / NB) * Np] = yi[e];
        __syncthreads();
    }
    for (int e = threadIdx.x; e < NB * nq; e += WG) s.Z[k * NB + e % NB + (q0 + e / NB) * Np] = zk[e];
}

// Back-substitution, part 1: x_k = D_k^{-1} z_k (D_k = U or R of step k).
template <int NB>
static __global__ __launch_bounds__(WG) void k_bwd_a(Ctx c, SolveArgs s, int k) {
    if (gated(s.gate)) return;
    __shared__ double zs[NB * RQ];
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    const double *Di = c.Dinv + (size_t)k * NB * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) zs[e] = s.Z[k * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    for (int e = threadIdx.x; e < NB * nq; e += WG) {
        int r = e % NB, q = e / NB;
        double acc = 0.0;
        for (int cc = r; cc < NB; ++cc) acc += Di[r + (size_t)cc * NB] * zs[q * NB + cc];
        s.X[k * NB + r + (q0 + q) * Np] = acc;
    }
}

// Back-substitution, part 2: z_i -= U_ik x_k for i < k.
template <int NB, class S>
static __global__ __launch_bounds__(WG) void k_bwd_b(Ctx c, SolveArgs s, int k) {
    if (gated(s.gate)) return;
    __shared__ double xs[NB * RQ];
    const int i = blockIdx.x;
    const int q0 = blockIdx.y * RQ, nq = min(RQ, s.nrhs - q0);
    const int64_t Np = c.n * NB;
    for (int e = threadIdx.x; e < NB * nq; e += WG) xs[e] = s.X[k * NB + e % NB + (q0 + e / NB) * Np];
    __syncthreads();
    const S *U = (const S *)c.At + c.toff(i, k);
    for (int r = threadIdx.x; r < NB; r += WG) {
        double acc[RQ];
        for (int q = 0; q < RQ; ++q) acc[q] = 0.0;
        for (int cc = 0; cc < NB; ++cc) {
            double a = (double)U[r + cc * NB];
#pragma unroll
            for (int q = 0; q < RQ; ++q)
                if (q < nq) acc[q] += a * xs[q * NB + cc];
        }
#pragma unroll
        for (int q = 0; q < RQ; ++q)
            if (q < nq) s.Z[i * NB + r + (q0 + q) * Np] -= acc[q];
    }
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

// Column-major FP64 A (lda) -> tile-major storage with identity padding.
template <class S>
static __global__ void k_to_tiles(const double *A, int64_t lda, int64_t N, int64_t n, int nb, S *At) {
    const int64_t Np = n * nb;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Np * Np) return;
    const int64_t tile = t / ((int64_t)nb * nb), e = t % ((int64_t)nb * nb);
    const int64_t i = tile % n, j = tile / n;
    const int64_t r = i * nb + e % nb, cc = j * nb + e / nb;
    double v = (r < N && cc < N) ? A[r + cc * lda] : (r == cc ? 1.0 : 0.0);
    At[t] = (S)v;
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
