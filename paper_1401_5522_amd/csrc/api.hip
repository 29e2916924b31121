// C ABI of the hybrid LU-QR solver (declarations and contracts in luqr.h).
#include <math.h>
#include <cmath>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "engine.h"
#include "krylov.h"

using namespace lq;

struct luqr_factors_s {
    Layout L;
    Ctx c;
    const Ops *ops;
    void *base;
    hipStream_t stream;
    luqr_opts o;
    int nsteps;
    std::vector<hipEvent_t> ev;  // LUQR_NPHASE + 1 per step when opts.timing is set
    std::vector<int> hdec;       // decision sequence, read once by the first GMRES refinement
    Side side{nullptr, nullptr, nullptr, nullptr, nullptr};  // lookahead stream and events (unless opts.no_lookahead)
};

static int hip_rc(hipError_t e) { return e == hipSuccess ? 0 : LUQR_ERR_HIP - (int)e; }


// The decisions are final once the factorization is done; GMRES refinement
// (which waits on the host anyway) reads them once and keeps them, so its
// solves launch only the kernels of the branch every step took.
static int host_decisions(luqr_factors f, const int **out) {
    if (f->hdec.empty()) {
        std::vector<int> d((size_t)f->L.n);
        hipError_t e = hipStreamSynchronize(f->stream);
        if (e == hipSuccess)
            e = hipMemcpy(d.data(), (char *)f->base + f->L.off_dec, d.size() * sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_rc(e);
        f->hdec.swap(d);
    }
    *out = f->hdec.data();
    return 0;
}

static const Ops *pick_ops(int nb, int prec) {
    switch (prec) {
    case LUQR_FP64: return ops_nb<P64>(nb);
    case LUQR_FP32: return ops_nb<P32>(nb);
    case LUQR_BF16: return ops_nb<PB16>(nb);
    default: return nullptr;
    }
}

// Validate options; returns 0 or the negative code of the offending argument
// position `pos_opts` (the opts pointer is one argument).
static int check_opts(int64_t N, const luqr_opts *o, int pos_opts) {
    if (!o) return -pos_opts;
    if (o->nb < 1) return -pos_opts;
    if (!(o->alpha >= 0.0)) return -pos_opts;
    if (o->criterion < 0 || o->criterion > 4) return -pos_opts;
    if (o->precision < 0 || o->precision > 2) return -pos_opts;
    if (o->criterion == LUQR_CRIT_FORCED && !o->forced) return -pos_opts;
    if (o->domain_stride < 0) return -pos_opts;
    if (o->invnorm_estimate < 0 || o->invnorm_estimate > 1) return -pos_opts;
    if (o->lu_variant < 0 || o->lu_variant > 2) return -pos_opts;
    if (o->qr_tree < 0) return -pos_opts;
    if (o->lu_variant == 2 && (o->criterion == LUQR_CRIT_MUMPS || o->domain_stride > 0 || o->invnorm_estimate))
        return LUQR_ERR_UNSUPPORTED;  // A2 has no GEPP pivots, domain or triangular L^-1 for these
    if (!pick_ops(o->nb, o->precision)) return LUQR_ERR_UNSUPPORTED;
    if (o->domain_stride > 0) {  // the domain's GEPP holds at most 512 stacked rows in one workgroup
        const int64_t n = (N + o->nb - 1) / o->nb;
        if ((1 + (n - 1) / o->domain_stride) * (int64_t)o->nb > 512) return LUQR_ERR_UNSUPPORTED;
    }
    return 0;
}

extern "C" int64_t luqr_workspace_bytes(int64_t N, const luqr_opts *o) {
    if (N < 1) return -1;
    int rc = check_opts(N, o, 2);
    if (rc) return rc;
    Layout L = make_layout(N, o->nb, o->precision, o->nrhs_max, o->domain_stride, o->qr_tree);
    return (int64_t)L.total;
}


extern "C" int luqr_factor(int64_t N, const double *dA, int64_t lda, const luqr_opts *o, void *dWork,
                           int64_t work_bytes, void *stream, luqr_factors *out) {
    if (N < 1) return -1;
    if (!dA) return -2;
    if (lda < N) return -3;
    int rc = check_opts(N, o, 4);
    if (rc) return rc;
    if (!dWork || ((uintptr_t)dWork & 255)) return -5;
    if (!out) return -8;
    Layout L = make_layout(N, o->nb, o->precision, o->nrhs_max, o->domain_stride, o->qr_tree);
    if (work_bytes < (int64_t)L.total) return -6;
    luqr_factors_s *f = new (std::nothrow) luqr_factors_s;
    if (!f) return LUQR_ERR_HIP - (int)hipErrorOutOfMemory;
    f->L = L;
    f->c = make_ctx(L, dWork, o->lu_variant == 2);
    f->ops = pick_ops(o->nb, o->precision);
    f->base = dWork;
    f->stream = (hipStream_t)stream;
    f->o = *o;
    f->o.forced = nullptr;
    f->nsteps = (o->nsteps < 0 || o->nsteps > L.n) ? (int)L.n : o->nsteps;
    if (o->timing) {
        f->ev.resize((size_t)(LUQR_NPHASE + 1) * f->nsteps);
        for (auto &e : f->ev) {
            hipError_t he = hipEventCreate(&e);
            if (he != hipSuccess) { e = nullptr; luqr_destroy(f); return hip_rc(he); }
        }
    }
    if (!o->no_lookahead) {
        hipError_t he = hipStreamCreateWithFlags(&f->side.st, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipStreamCreateWithFlags(&f->side.st2, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&f->side.ea, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&f->side.eb, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&f->side.el, hipEventDisableTiming);
        if (he != hipSuccess) { luqr_destroy(f); return hip_rc(he); }
    }
    (void)hipGetLastError();
    f->ops->factor(f->c, L, dA, lda, *o, f->nsteps, f->stream, f->ev.empty() ? nullptr : f->ev.data(),
                   f->side.st ? &f->side : nullptr);
    rc = hip_rc(hipGetLastError());
    if (rc) { luqr_destroy(f); return rc; }
    *out = f;
    return 0;
}

static SolveArgs solve_args(const Layout &L, void *base, int nrhs, const int *gate) {
    char *b = (char *)base;
    SolveArgs s;
    s.Y = (double *)(b + L.off_Y);
    s.Z = (double *)(b + L.off_Z);
    s.X = (double *)(b + L.off_X);
    s.G = (double *)(b + L.off_G);
    s.nrhs = nrhs;
    s.gate = gate;
    return s;
}

extern "C" int luqr_solve(luqr_factors f, int64_t nrhs, double *dB, int64_t ldb, void *stream) {
    if (!f) return -1;
    if (nrhs < 1 || nrhs > f->L.nrhs_max) return -2;
    if (!dB) return -3;
    if (ldb < f->L.N) return -4;
    if (f->nsteps < f->L.n) return LUQR_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    SolveArgs s = solve_args(f->L, f->base, (int)nrhs, nullptr);
    (void)hipGetLastError();
    k_rhs_in<<<nblk(f->L.Np * nrhs), WG, 0, st>>>(dB, ldb, s.Y, f->L.N, f->L.Np, (int)nrhs, nullptr);
    f->ops->solve(f->c, f->L, s, nullptr, st);  // both branches per step, decided on the device
    k_rhs_out<<<nblk(f->L.N * nrhs), WG, 0, st>>>(s.X, dB, ldb, f->L.N, f->L.Np, (int)nrhs);
    return hip_rc(hipGetLastError());
}

// The body of luqr_solve_refined over a factorization in the workspace at
// `base`.  hdec: the decision sequence if the host holds it, else nullptr.
// Every iteration is enqueued; once the device test has passed, the kernels
// of the later ones return at once (they read the convergence flag), so
// nothing waits on the host.
static int refined_solve(const Layout &L, const Ctx &c, const Ops *ops, void *base, const int *hdec,
                         const double *dA, int64_t lda, int64_t nrhs, const double *dB, int64_t ldb, double *dX,
                         int64_t ldx, int32_t max_iter, hipStream_t st) {
    char *b = (char *)base;
    int *conv = (int *)(b + L.off_conv);
    double *R = (double *)(b + L.off_R);
    double *D = (double *)(b + L.off_D);
    double *Xk = (double *)(b + L.off_Xd);
    double *part = (double *)(b + L.off_part);
    double *norms = (double *)(b + L.off_rnorm);
    double *apart = (double *)(b + L.off_apart);
    const int nq = (int)nrhs;
    const int64_t total = L.Np * nrhs;
    (void)hipGetLastError();
    k_ir_reset<<<1, 64, 0, st>>>(c.st, conv);
    k_fill_f64<<<nblk(2 * nrhs + 1), WG, 0, st>>>(norms, 2 * nrhs + 1);  // ||r||, ||x|| per column, ||A||
    // x0 = solve(b): solve writes its result into X; keep the iterate in Xk
    SolveArgs s = solve_args(L, base, nq, nullptr);
    k_rhs_in<<<nblk(total), WG, 0, st>>>(dB, ldb, s.Y, L.N, L.Np, nq, nullptr);
    ops->solve(c, L, s, hdec, st);
    hipError_t ce = hipMemcpyAsync(Xk, s.X, total * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (ce != hipSuccess) return hip_rc(ce);
    const dim3 rgrid(nblk(L.N), (unsigned)L.nparts, (unsigned)((nq + RQR - 1) / RQR));
    const dim3 rgrid_final(nblk(L.N * nrhs));
    for (int it = 0; it <= max_iter; ++it) {
        const bool last = it == max_iter;
        k_resid_part<<<rgrid, WG, 0, st>>>(dA, lda, L.N, L.Np, Xk, nq, part, it == 0 ? apart : nullptr, conv);
        k_resid_final<<<rgrid_final, WG, 0, st>>>(dB, ldb, L.N, L.Np, nq, (int)L.nparts, part,
                                                  it == 0 ? apart : nullptr, Xk, R, norms, conv);
        k_ir_check<<<1, 64, 0, st>>>(norms, nq, L.N, conv, c.st, last ? 1 : 0);
        if (last) break;
        SolveArgs sr = solve_args(L, base, nq, conv);
        // rows N..Np-1 of R are never written by the residual kernels: copy
        // only the first N rows and zero the padding
        k_rhs_in<<<nblk(total), WG, 0, st>>>(R, L.Np, sr.Y, L.N, L.Np, nq, conv);
        sr.X = D;
        ops->solve(c, L, sr, hdec, st);
        k_ir_update<<<nblk(total), WG, 0, st>>>(Xk, D, total, conv);
    }
    k_rhs_out<<<nblk(L.N * nrhs), WG, 0, st>>>(Xk, dX, ldx, L.N, L.Np, nq);
    return hip_rc(hipGetLastError());
}


extern "C" int luqr_solve_refined(luqr_factors f, const double *dA, int64_t lda, int64_t nrhs, const double *dB,
                                  int64_t ldb, double *dX, int64_t ldx, int32_t max_iter, void *stream) {
    if (!f) return -1;
    if (!dA) return -2;
    if (lda < f->L.N) return -3;
    if (nrhs < 1 || nrhs > f->L.nrhs_max) return -4;
    if (!dB) return -5;
    if (ldb < f->L.N) return -6;
    if (!dX) return -7;
    if (ldx < f->L.N) return -8;
    if (max_iter < 0) return -9;
    if (f->nsteps < f->L.n) return LUQR_ERR_UNSUPPORTED;
    return refined_solve(f->L, f->c, f->ops, f->base, nullptr, dA, lda, nrhs, dB, ldb, dX, ldx, max_iter,
                         (hipStream_t)stream);
}

// GMRES-based iterative refinement (one right-hand side).  Outer loop in
// FP64: r = b - A x, the convergence test of luqr_solve_refined, and x += d
// where d solves A d = r by GMRES(m) in FP64, left-preconditioned by the
// stored factors (M^{-1} = the hybrid LU-QR solve): the Arnoldi basis is
// orthogonalized by classical Gram-Schmidt applied twice, the small
// Hessenberg least-squares problem is solved on the host with Givens
// rotations, and the inner loop stops when the preconditioned residual has
// dropped by GMRES_TOL or after max_inner vectors.  Every vector operation
// runs on the device; the host reads back j + 2 numbers per inner step.
constexpr double GMRES_TOL = 1e-6;

extern "C" int luqr_solve_gmres_ir(luqr_factors f, const double *dA, int64_t lda, const double *db, double *dx,
                                   int32_t max_outer, int32_t max_inner, int32_t *inner_total, void *stream) {
    if (!f) return -1;
    if (!dA) return -2;
    if (lda < f->L.N) return -3;
    if (!db) return -4;
    if (!dx) return -5;
    if (max_outer < 0) return -6;
    if (max_inner < 1 || max_inner > KRYLOV_MAX) return -7;
    if (f->nsteps < f->L.n) return LUQR_ERR_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    const Layout &L = f->L;
    const int *hdec;
    int rc0 = host_decisions(f, &hdec);
    if (rc0) return rc0;
    char *b = (char *)f->base;
    const int64_t N = L.N, Np = L.Np;
    int *conv = (int *)(b + L.off_conv);
    double *R = (double *)(b + L.off_R);      // residual, or -A v for a basis vector v
    double *Z0 = (double *)(b + L.off_D);     // zeros: the right-hand side of a plain product A v
    double *X = (double *)(b + L.off_Xd);     // iterate
    double *part = (double *)(b + L.off_part);
    double *apart = (double *)(b + L.off_apart);
    double *norms = (double *)(b + L.off_rnorm);
    double *V = (double *)(b + L.off_kry);    // basis V_0 .. V_m (Np apart)
    double *W = V + (size_t)(KRYLOV_MAX + 1) * Np;
    double *dpart = (double *)(b + L.off_kdots);
    double *h1 = dpart + (KRYLOV_MAX + 1) * DOT_BLOCKS;
    double *h2 = h1 + (KRYLOV_MAX + 1);
    double *nrm = h2 + (KRYLOV_MAX + 1);
    double *ycoef = nrm + 2;
    const unsigned vb = nblk(Np);
    const dim3 rgrid(nblk(N), (unsigned)L.nparts, 1);
    const dim3 rgrid_final(nblk(N));
    SolveArgs s = solve_args(f->L, f->base, 1, nullptr);
    hipError_t e = hipSuccess;
    auto precond = [&](const double *src, int64_t ld, double *dst) {  // dst = M^{-1} src
        k_rhs_in<<<vb, WG, 0, st>>>(src, ld, s.Y, N, Np, 1, nullptr);
        f->ops->solve(f->c, L, s, hdec, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dst, s.X, Np * sizeof(double), hipMemcpyDeviceToDevice, st);
    };
    auto dots = [&](const double *Vb, int nv, const double *w, double *out) {  // out[i] = V_i . w
        k_dots_part<<<dim3(DOT_BLOCKS, nv), WG, 0, st>>>(Vb, Np, w, Np, dpart);
        k_dots_final<<<1, 64, 0, st>>>(dpart, nv, out);
    };
    auto fetch = [&](double *host, const double *dev, size_t count) {
        if (e == hipSuccess) e = hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    };
    (void)hipGetLastError();
    k_ir_reset<<<1, 64, 0, st>>>(f->c.st, conv);
    k_fill_f64<<<1, 64, 0, st>>>(norms, 3);
    k_fill_f64<<<vb, WG, 0, st>>>(Z0, Np);
    precond(db, N, X);  // x_0 = M^{-1} b
    const int m = max_inner;
    std::vector<double> Hc((size_t)m * (m + 1)), g(m + 1), cs(m), sn(m), y(m), hb(2 * (KRYLOV_MAX + 1) + 1);
    int inner = 0;
    for (int outer = 0;; ++outer) {
        const bool last = outer == max_outer;
        k_fill_f64<<<1, 64, 0, st>>>(norms, 2);  // keep ||A|| (slot 2) once known
        k_resid_part<<<rgrid, WG, 0, st>>>(dA, lda, N, Np, X, 1, part, outer == 0 ? apart : nullptr, nullptr);
        k_resid_final<<<rgrid_final, WG, 0, st>>>(db, N, N, Np, 1, (int)L.nparts, part,
                                                  outer == 0 ? apart : nullptr, X, R, norms, nullptr);
        k_ir_check<<<1, 64, 0, st>>>(norms, 1, N, conv, f->c.st, last ? 1 : 0);
        int done = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&done, conv, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_rc(e);
        if (done || last) break;
        // GMRES(m) on M^{-1} A d = M^{-1} r
        precond(R, Np, V);
        dots(V, 1, V, nrm);
        double beta2 = 0.0;
        fetch(&beta2, nrm, 1);
        if (e != hipSuccess) return hip_rc(e);
        if (!(beta2 > 0.0)) break;
        const double beta = sqrt(beta2);
        k_normalize<<<vb, WG, 0, st>>>(V, V, nrm, Np);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int used = 0;
        for (int j = 0; j < m; ++j) {
            double *Vj = V + (size_t)j * Np;
            k_resid_part<<<rgrid, WG, 0, st>>>(dA, lda, N, Np, Vj, 1, part, nullptr, nullptr);
            k_resid_final<<<rgrid_final, WG, 0, st>>>(Z0, Np, N, Np, 1, (int)L.nparts, part, nullptr, Vj, R, norms,
                                                      nullptr);                      // R = -A V_j
            precond(R, Np, W);                                                   // W = -M^{-1} A V_j
            k_lincomb<<<vb, WG, 0, st>>>(W, -1.0, V, Np, 0, nullptr, 0.0, Np);   // w = M^{-1} A V_j
            dots(V, j + 1, W, h1);                                               // two Gram-Schmidt passes
            k_lincomb<<<vb, WG, 0, st>>>(W, 1.0, V, Np, j + 1, h1, -1.0, Np);
            dots(V, j + 1, W, h2);
            k_lincomb<<<vb, WG, 0, st>>>(W, 1.0, V, Np, j + 1, h2, -1.0, Np);
            dots(W, 1, W, nrm);
            fetch(hb.data(), h1, 2 * (KRYLOV_MAX + 1) + 1);  // h1, h2, |w|^2 are contiguous
            if (e != hipSuccess) return hip_rc(e);
            double *hc = &Hc[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) hc[i] = hb[i] + hb[KRYLOV_MAX + 1 + i];
            const double hn2 = hb[2 * (KRYLOV_MAX + 1)];
            const double hnext = hn2 > 0.0 ? sqrt(hn2) : 0.0;
            for (int i = 0; i < j; ++i) {  // earlier rotations
                const double a0 = cs[i] * hc[i] + sn[i] * hc[i + 1];
                hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
                hc[i] = a0;
            }
            const double rr = hypot(hc[j], hnext);
            cs[j] = rr > 0.0 ? hc[j] / rr : 1.0;
            sn[j] = rr > 0.0 ? hnext / rr : 0.0;
            hc[j] = rr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            used = j + 1;
            if (!(hnext > 0.0) || fabs(g[j + 1]) <= GMRES_TOL * beta) break;
            if (j + 1 < m) k_normalize<<<vb, WG, 0, st>>>(V + (size_t)(j + 1) * Np, W, nrm, Np);
        }
        inner += used;
        for (int i = used - 1; i >= 0; --i) {  // y = H^{-1} g (upper triangular after the rotations)
            double acc = g[i];
            for (int k2 = i + 1; k2 < used; ++k2) acc -= Hc[(size_t)k2 * (m + 1) + i] * y[k2];
            y[i] = Hc[(size_t)i * (m + 1) + i] != 0.0 ? acc / Hc[(size_t)i * (m + 1) + i] : 0.0;
        }
        if (e == hipSuccess) e = hipMemcpyAsync(ycoef, y.data(), used * sizeof(double), hipMemcpyHostToDevice, st);
        k_lincomb<<<vb, WG, 0, st>>>(X, 1.0, V, Np, used, ycoef, 1.0, Np);  // x += V y
        if (e == hipSuccess) e = hipStreamSynchronize(st);  // y is read before it goes out of scope
        if (e != hipSuccess) return hip_rc(e);
    }
    if (inner_total) *inner_total = inner;
    k_rhs_out<<<nblk(N), WG, 0, st>>>(X, dx, N, N, Np, 1);
    return hip_rc(hipGetLastError());
}

extern "C" double luqr_alpha_for_growth(int64_t N, int32_t nb, int32_t criterion, double growth) {
    if (N < 1 || nb < 1) return -1.0;
    if (criterion != LUQR_CRIT_MAX && criterion != LUQR_CRIT_SUM) return -3.0;
    if (!(growth >= 1.0)) return -4.0;
    const int64_t n = (N + nb - 1) / nb;
    if (n == 1) return INFINITY;
    const double e = 1.0 / (double)(n - 1);
    if (criterion == LUQR_CRIT_MAX) return std::pow(growth, e) - 1.0;  // (1 + alpha)^(n-1) = growth
    if (growth < (double)n) return 0.0;                                // the Sum bound is n at best
    return std::pow(growth / (double)n, e);                            // n alpha^(n-1) = growth
}

extern "C" int luqr_get_decisions(luqr_factors f, int8_t *dec, double *s, double *m, double *margin, int64_t n) {
    if (!f) return -1;
    if (n < 0 || n > f->L.n) return -6;
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_rc(e);
    char *b = (char *)f->base;
    if (dec) {
        int tmp[4096];
        for (int64_t k0 = 0; k0 < n; k0 += 4096) {
            int64_t cnt = n - k0 < 4096 ? n - k0 : 4096;
            e = hipMemcpy(tmp, (int *)(b + f->L.off_dec) + k0, cnt * sizeof(int), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_rc(e);
            for (int64_t q = 0; q < cnt; ++q) dec[k0 + q] = (int8_t)tmp[q];
        }
    }
    if (s && (e = hipMemcpy(s, b + f->L.off_s, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return hip_rc(e);
    if (m && (e = hipMemcpy(m, b + f->L.off_m, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return hip_rc(e);
    if (margin && (e = hipMemcpy(margin, b + f->L.off_margin, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_rc(e);
    return 0;
}

extern "C" int luqr_get_status(luqr_factors f, luqr_status *st) {
    if (!f) return -1;
    if (!st) return -2;
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_rc(e);
    DevStatus d;
    e = hipMemcpy(&d, (char *)f->base + f->L.off_status, sizeof(d), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_rc(e);
    st->info = d.info;
    st->nonfinite = d.nonfinite;
    st->n_lu = d.n_lu;
    st->ir_iters = d.ir_iters;
    st->ir_converged = d.ir_converged;
    st->ir_eta = d.ir_eta;
    st->watchdog = d.watchdog;
    st->reserved = 0;
    return 0;
}

extern "C" int luqr_export_factors(luqr_factors f, double *dF, int64_t ldf, int32_t *ipiv, void *stream) {
    if (!f) return -1;
    if (!dF) return -2;
    if (ldf < f->L.N) return -3;
    hipStream_t st = (hipStream_t)stream;
    (void)hipGetLastError();
    f->ops->export_factors(f->c, f->L, dF, ldf, st);
    int rc = hip_rc(hipGetLastError());
    if (rc || !ipiv) return rc;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_rc(e);
    const int64_t n = f->L.n, nb = f->L.nb, N = f->L.N;
    char *b = (char *)f->base;
    int *dev_ipiv = (int *)(b + f->L.off_ipiv);
    int *dev_dec = (int *)(b + f->L.off_dec);
    for (int64_t k = 0; k < n; ++k) {
        int d = 0;
        e = hipMemcpy(&d, dev_dec + k, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_rc(e);
        const int64_t mk = (k < n - 1) ? nb : N - (n - 1) * nb;
        if (d == 1) {
            e = hipMemcpy(ipiv + k * nb, dev_ipiv + k * nb, mk * sizeof(int), hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_rc(e);
        } else {
            for (int64_t c = 0; c < mk; ++c) ipiv[k * nb + c] = (int32_t)c;
        }
    }
    return 0;
}

extern "C" int luqr_get_step_times(luqr_factors f, float *t, int64_t n) {
    if (!f) return -1;
    if (!t) return -2;
    if (n < 0 || n > f->nsteps) return -3;
    if (f->ev.empty()) return LUQR_ERR_UNSUPPORTED;
    hipError_t e = hipStreamSynchronize(f->stream);
    if (e != hipSuccess) return hip_rc(e);
    for (int64_t k = 0; k < n; ++k) {
        hipEvent_t *v = &f->ev[(size_t)(LUQR_NPHASE + 1) * k];
        for (int p = 0; p < LUQR_NPHASE; ++p)
            if ((e = hipEventElapsedTime(&t[LUQR_NPHASE * k + p], v[p], v[p + 1])) != hipSuccess) return hip_rc(e);
    }
    return 0;
}

extern "C" void luqr_destroy(luqr_factors f) {
    if (!f) return;
    for (auto &e : f->ev)
        if (e) (void)hipEventDestroy(e);
    if (f->side.st) {
        (void)hipStreamSynchronize(f->side.st);  // its work was joined to the caller's stream
        (void)hipStreamDestroy(f->side.st);
    }
    if (f->side.st2) {
        (void)hipStreamSynchronize(f->side.st2);
        (void)hipStreamDestroy(f->side.st2);
    }
    if (f->side.ea) (void)hipEventDestroy(f->side.ea);
    if (f->side.eb) (void)hipEventDestroy(f->side.eb);
    if (f->side.el) (void)hipEventDestroy(f->side.el);
    delete f;
}


// ---- the entry point that allocates nothing ---------------------------------
// luqr_solve_noalloc takes its workspace from `scratch`, a file-scope device
// array.  Each GPU the library runs on holds its own copy until the process
// ends.  In host code the array's name is only a stand-in for the symbol, not
// a device address: the address of the current GPU's copy is looked up once
// per device with hipGetSymbolAddress and kept in g_scratch_ptr, and only that
// pointer is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[LUQR_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr int NOALLOC_MAX_STEPS = 1024;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

static int scratch_for_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_rc(e);
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LUQR_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_rc(e);
        if (!p || ((uintptr_t)p & 255)) return LUQR_ERR_HIP - (int)hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

extern "C" int luqr_solve_noalloc(int64_t N, const double *dA, int64_t lda, const luqr_opts *o, int64_t nrhs,
                                  const double *dB, int64_t ldb, double *dX, int64_t ldx, int32_t max_iter,
                                  luqr_status *status, void *stream) {
    if (N < 1) return -1;
    if (!dA) return -2;
    if (lda < N) return -3;
    int rc = check_opts(N, o, 4);
    if (rc) return rc;
    if (o->timing) return -4;                      // events would have to be created
    if (nrhs < 1 || nrhs > o->nrhs_max) return -5;
    if (!dB) return -6;
    if (ldb < N) return -7;
    if (!dX) return -8;
    if (ldx < N) return -9;
    if (max_iter < 0) return -10;
    const Layout L = make_layout(N, o->nb, o->precision, o->nrhs_max, o->domain_stride, o->qr_tree);
    if (o->nsteps >= 0 && o->nsteps < L.n) return -4;   // a partial factorization cannot be solved with
    if (L.total > (size_t)LUQR_NOALLOC_SCRATCH_BYTES || L.n > NOALLOC_MAX_STEPS) return LUQR_ERR_TOO_LARGE;
    void *base = nullptr;
    rc = scratch_for_current_device(&base);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Ctx c = make_ctx(L, base, o->lu_variant == 2);
    const Ops *ops = pick_ops(o->nb, o->precision);
    luqr_opts oo = *o;
    oo.no_lookahead = 1;                           // one stream: no side stream to create
    (void)hipGetLastError();
    ops->factor(c, L, dA, lda, oo, (int)L.n, st, nullptr, nullptr);
    rc = hip_rc(hipGetLastError());
    if (rc) return rc;
    rc = refined_solve(L, c, ops, base, nullptr, dA, lda, nrhs, dB, ldb, dX, ldx, max_iter, st);
    if (rc || !status) return rc;
    DevStatus d;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(&d, (char *)base + L.off_status, sizeof(d), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_rc(e);
    status->info = d.info;
    status->nonfinite = d.nonfinite;
    status->n_lu = d.n_lu;
    status->ir_iters = d.ir_iters;
    status->ir_converged = d.ir_converged;
    status->ir_eta = d.ir_eta;
    status->watchdog = d.watchdog;
    status->reserved = 0;
    return 0;
}
