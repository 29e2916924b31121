// C ABI of the hybrid LU-QR solver (declarations and contracts in luqr.h).
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "engine.h"

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
    std::vector<int> hdec;       // decision sequence, read once by the first solve
    Side side{nullptr, nullptr, nullptr};  // lookahead stream and events (unless opts.no_lookahead)
};

static int hip_rc(hipError_t e) { return e == hipSuccess ? 0 : LUQR_ERR_HIP - (int)e; }


// The decisions are final once the factorization is done; the first solve
// waits for it once and keeps them, so each later solve launches only the
// kernels of the branch every step took.
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
    if (o->mumps_reading < 0 || o->mumps_reading > 2) return -pos_opts;
    if (!pick_ops(o->nb, o->precision)) return LUQR_ERR_UNSUPPORTED;
    (void)N;
    return 0;
}

extern "C" int64_t luqr_workspace_bytes(int64_t N, const luqr_opts *o) {
    if (N < 1) return -1;
    int rc = check_opts(N, o, 2);
    if (rc) return rc;
    Layout L = make_layout(N, o->nb, o->precision, o->nrhs_max);
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
    Layout L = make_layout(N, o->nb, o->precision, o->nrhs_max);
    if (work_bytes < (int64_t)L.total) return -6;
    luqr_factors_s *f = new (std::nothrow) luqr_factors_s;
    if (!f) return LUQR_ERR_HIP - (int)hipErrorOutOfMemory;
    f->L = L;
    f->c = make_ctx(L, dWork);
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
        if (he == hipSuccess) he = hipEventCreateWithFlags(&f->side.ea, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&f->side.eb, hipEventDisableTiming);
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

static SolveArgs solve_args(luqr_factors f, int nrhs, const int *gate) {
    char *b = (char *)f->base;
    SolveArgs s;
    s.Y = (double *)(b + f->L.off_Y);
    s.Z = (double *)(b + f->L.off_Z);
    s.X = (double *)(b + f->L.off_X);
    s.G = (double *)(b + f->L.off_G);
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
    const int *hdec;
    int rc = host_decisions(f, &hdec);
    if (rc) return rc;
    SolveArgs s = solve_args(f, (int)nrhs, nullptr);
    (void)hipGetLastError();
    k_rhs_in<<<nblk(f->L.Np * nrhs), WG, 0, st>>>(dB, ldb, s.Y, f->L.N, f->L.Np, (int)nrhs, nullptr);
    f->ops->solve(f->c, f->L, s, hdec, st);
    k_rhs_out<<<nblk(f->L.N * nrhs), WG, 0, st>>>(s.X, dB, ldb, f->L.N, f->L.Np, (int)nrhs);
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
    hipStream_t st = (hipStream_t)stream;
    const Layout &L = f->L;
    const int *hdec;
    int rc0 = host_decisions(f, &hdec);
    if (rc0) return rc0;
    char *b = (char *)f->base;
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
    k_ir_reset<<<1, 64, 0, st>>>(f->c.st, conv);
    k_fill_f64<<<nblk(2 * nrhs + 1), WG, 0, st>>>(norms, 2 * nrhs + 1);  // ||r||, ||x|| per column, ||A||
    // x0 = solve(b): solve writes its result into X; keep the iterate in Xk
    SolveArgs s = solve_args(f, nq, nullptr);
    k_rhs_in<<<nblk(total), WG, 0, st>>>(dB, ldb, s.Y, L.N, L.Np, nq, nullptr);
    f->ops->solve(f->c, L, s, hdec, st);
    hipError_t ce = hipMemcpyAsync(Xk, s.X, total * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (ce != hipSuccess) return hip_rc(ce);
    const dim3 rgrid(nblk(L.N), (unsigned)L.nparts, (unsigned)((nq + RQR - 1) / RQR));
    const dim3 rgrid_final(nblk(L.N * nrhs));
    for (int it = 0; it <= max_iter; ++it) {
        const bool last = it == max_iter;
        k_resid_part<<<rgrid, WG, 0, st>>>(dA, lda, L.N, L.Np, Xk, nq, part, it == 0 ? apart : nullptr, conv);
        k_resid_final<<<rgrid_final, WG, 0, st>>>(dB, ldb, L.N, L.Np, nq, (int)L.nparts, part,
                                                  it == 0 ? apart : nullptr, Xk, R, norms, conv);
        k_ir_check<<<1, 64, 0, st>>>(norms, nq, L.N, conv, f->c.st, last ? 1 : 0);
        if (last) break;
        // stop enqueuing once the test has passed (one small read per iteration)
        int done = 0;
        hipError_t ce2 = hipMemcpyAsync(&done, conv, sizeof(int), hipMemcpyDeviceToHost, st);
        if (ce2 == hipSuccess) ce2 = hipStreamSynchronize(st);
        if (ce2 != hipSuccess) return hip_rc(ce2);
        if (done) break;
        SolveArgs sr = solve_args(f, nq, conv);
        k_rhs_in<<<nblk(total), WG, 0, st>>>(R, L.Np, sr.Y, L.Np, L.Np, nq, conv);
        sr.X = D;
        f->ops->solve(f->c, L, sr, hdec, st);
        k_ir_update<<<nblk(total), WG, 0, st>>>(Xk, D, total, conv);
    }
    k_rhs_out<<<nblk(L.N * nrhs), WG, 0, st>>>(Xk, dX, ldx, L.N, L.Np, nq);
    return hip_rc(hipGetLastError());
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
    if (f->side.ea) (void)hipEventDestroy(f->side.ea);
    if (f->side.eb) (void)hipEventDestroy(f->side.eb);
    delete f;
}

