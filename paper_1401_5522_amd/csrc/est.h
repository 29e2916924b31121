// O(n_b^2)-per-iteration estimate of ||A_kk^{-1}||_1 for the Max and Sum
// criteria (Sec. 3.4: the norm can be approximated from the L and U factors
// by an iterative method), the option opts.invnorm_estimate.
#pragma once
#include "solve.h"

namespace lq {

// Hager's iteration with Higham's refinements (the one LAPACK's condition
// estimator runs), on B = U^{-1} L^{-1}: the inverse of P A_kk up to a
// column permutation, which leaves the 1-norm unchanged.  Products with B
// and B^T go through the explicit FP64 inverses k_panel_trtri formed, two
// tile-vector products each.  Over the mk real columns of the tile (the
// padding is an identity block and stays out of every vector):
//   x = 1/mk; y = B x; est = |y|_1; xi = sign(y); z = B^T xi;
//   up to four times: j = the first index of max |z|; y = B e_j; est = |y|_1;
//   stop if sign(y) repeats xi or est did not grow (the new value stands);
//   else xi = sign(y), z = B^T xi, and stop once z_jlast == max |z|;
//   finally est = max(est, 2 |B x|_1 / (3 mk)) with x_i = (-1)^i (1 + i/(mk-1)).
// sign(0) = +1.  One workgroup; the estimate goes to the decision through
// the inverse-norm partial sums (column 0 holds it, the others zero).
template <int NB>
__global__ __launch_bounds__(WG) void k_panel_invest(Ctx c, int k) {
    constexpr int RB = mv_rb<NB>(), NRB = NB / RB;
    __shared__ double xv[NB], tv[NB], yv[NB];
    __shared__ double red[4 * 1 * 64];
    __shared__ double dsum[WG];
    __shared__ int isg[NB], iarg[WG], ok[WG];
    const int tid = threadIdx.x, l = lane_id(), w = wave_id();
    const int mk = c.msize(k);
    const double *Ui = c.Dinv + (size_t)k * NB * NB;
    const double *Li = c.Linv + (size_t)k * NB * NB;
    // y = B v = U^{-1} (L^{-1} v) (v in xv, result in yv)
    auto apply = [&]() {
        double out[1];
        for (int rb = 0; rb < NRB; ++rb) {
            if (rows_mv<NB, 2, double, 1>(Li, xv, 1, rb * RB, out, red)) tv[rb * RB + l] = out[0];
            __syncthreads();
        }
        for (int rb = 0; rb < NRB; ++rb) {
            if (rows_mv<NB, 1, double, 1>(Ui, tv, 1, rb * RB, out, red)) yv[rb * RB + l] = out[0];
            __syncthreads();
        }
    };
    // z = B^T v = L^{-T} (U^{-T} v) (v in xv, result in yv)
    auto apply_t = [&]() {
        cols_dot<NB, WG / 64, 1, double>(Ui, xv, 1, tv, NB, 0, NB);
        __syncthreads();
        cols_dot<NB, WG / 64, 2, double>(Li, tv, 1, yv, NB, 0, NB);
        __syncthreads();
    };
    auto norm1 = [&]() {  // |yv|_1 over the real rows
        double s = 0.0;
        for (int i = tid; i < mk; i += WG) s += fabs(yv[i]);
        dsum[tid] = s;
        __syncthreads();
        double t = 0.0;
        for (int u = 0; u < WG; ++u) t += dsum[u];
        __syncthreads();
        return t;
    };
    auto argmax = [&]() {  // first index of max |yv| over the real rows
        double b = -1.0;
        int bi = 0;
        for (int i = tid; i < mk; i += WG)
            if (fabs(yv[i]) > b) { b = fabs(yv[i]); bi = i; }
        dsum[tid] = b;
        iarg[tid] = bi;
        __syncthreads();
        double bb = dsum[0];
        int bj = iarg[0];
        for (int u = 1; u < WG; ++u)
            if (dsum[u] > bb || (dsum[u] == bb && iarg[u] < bj)) { bb = dsum[u]; bj = iarg[u]; }
        __syncthreads();
        return bj;
    };
    auto set_x = [&](auto f) {
        for (int i = tid; i < NB; i += WG) xv[i] = i < mk ? f(i) : 0.0;
        __syncthreads();
    };
    set_x([&](int) { return 1.0 / (double)mk; });
    apply();
    double est = norm1();
    if (mk > 1) {
        for (int i = tid; i < NB; i += WG) {
            isg[i] = yv[i] >= 0.0 ? 1 : -1;
            xv[i] = i < mk ? (double)isg[i] : 0.0;
        }
        __syncthreads();
        apply_t();
        int j = argmax();
        for (int iter = 2;; ++iter) {
            set_x([&](int i) { return i == j ? 1.0 : 0.0; });
            apply();
            const double estold = est;
            est = norm1();
            int same = 1;
            for (int i = tid; i < mk; i += WG) same &= ((yv[i] >= 0.0 ? 1 : -1) == isg[i]);
            ok[tid] = same;
            __syncthreads();
            for (int u = 0; u < WG; ++u) same &= ok[u];
            __syncthreads();
            if (same || est <= estold) break;
            for (int i = tid; i < NB; i += WG) {
                isg[i] = yv[i] >= 0.0 ? 1 : -1;
                xv[i] = i < mk ? (double)isg[i] : 0.0;
            }
            __syncthreads();
            apply_t();
            const int jlast = j;
            j = argmax();
            if (yv[jlast] == fabs(yv[j]) || iter >= 5) break;
        }
        set_x([&](int i) { return (i % 2 ? -1.0 : 1.0) * (1.0 + (double)i / (double)(mk - 1)); });
        apply();
        const double alt = 2.0 * norm1() / (3.0 * (double)mk);
        if (alt > est) est = alt;
    }
    for (int rb = 0; rb < (NB < 64 ? 1 : NB / 64); ++rb)
        for (int jj = tid; jj < NB; jj += WG) c.invpart[(size_t)rb * NB + jj] = (rb == 0 && jj == 0) ? est : 0.0;
}

}  // namespace lq
