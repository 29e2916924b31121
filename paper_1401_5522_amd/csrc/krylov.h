// Vector kernels of GMRES-based iterative refinement (luqr_solve_gmres_ir):
// the outer loop refines x in FP64 with the residual kernels of the solve
// path; each correction A d = r is found by FP64 GMRES preconditioned with the
// stored (storage-precision) factors, x_0 = M^{-1} b, M^{-1} = the hybrid
// LU-QR solve.  Vectors are FP64 of np entries (the padded size; padding
// entries stay zero).  Reductions are two-pass in a fixed order, so a run
// is reproducible.
#pragma once
#include "common.h"

namespace lq {

constexpr int DOT_BLOCKS = 64;  // partial sums per dot product

// part[i * DOT_BLOCKS + blk] = sum over this block's rows of V_i[r] w[r],
// i < nv (grid: DOT_BLOCKS x nv).
static __global__ __launch_bounds__(WG) void k_dots_part(const double *V, int64_t ldv, const double *w, int64_t np,
                                                         double *part) {
    __shared__ double red[WG / 64];
    const int i = blockIdx.y;
    const double *v = V + (int64_t)i * ldv;
    double s = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * WG + threadIdx.x; r < np; r += (int64_t)DOT_BLOCKS * WG) s += v[r] * w[r];
    s = wave_sum(s);
    if (lane_id() == 0) red[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[i * DOT_BLOCKS + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dots[i] = sum of the partials of dot i, in block order (one thread each).
static __global__ void k_dots_final(const double *part, int nv, double *dots) {
    const int i = threadIdx.x;
    if (i >= nv) return;
    double s = 0.0;
    for (int b = 0; b < DOT_BLOCKS; ++b) s += part[i * DOT_BLOCKS + b];
    dots[i] = s;
}

// w[r] = a w[r] + sign sum_{i < nv} coef[i] V_i[r]   (coef in device memory).
static __global__ void k_lincomb(double *w, double a, const double *V, int64_t ldv, int nv, const double *coef,
                                 double sign, int64_t np) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= np) return;
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s += coef[i] * V[(int64_t)i * ldv + r];
    w[r] = a * w[r] + sign * s;
}

// out[r] = in[r] / sqrt(*nrm2)   (in-place allowed).
static __global__ void k_normalize(double *out, const double *in, const double *nrm2, int64_t np) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= np) return;
    out[r] = in[r] / sqrt(*nrm2);
}

}  // namespace lq
