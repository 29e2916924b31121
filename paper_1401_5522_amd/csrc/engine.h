// Host-side launch sequences.  The host enqueues every kernel of every step
// without waiting (on one stream, or two with lookahead): the LU-or-QR decision of step k is written
// to device memory by k_panel_decide and both branch kernels read it there,
// returning at once when they are not the chosen branch (the dynamic task
// graph of Sec. 4 without a host round trip).
#pragma once
#include "lu.h"
#include "panel.h"
#include "qr.h"
#include "solve.h"
#include "est.h"

namespace lq {

// Panel of variant A2 (Sec. 2.3): GEQRT of the FP64 copy W_k of A_kk by the
// QR step's producers in FP64 (workgroups 0..nb/IB-1), T's diagonal blocks
// into the Dinv_k slot until k_a2_commit; publishes the flags of tile k for
// the QR step that may continue from it.  The criterion's tile norms run
// beside it (the workgroups after the producers, tile k+1.. in order).
template <int NB, class S>
__global__ __launch_bounds__(WG) void k_a2_geqrt(Ctx c, int k) {
    __shared__ __attribute__((aligned(16))) char smem[qr_lds<NB, P64>()];
    if ((int)blockIdx.x >= qr_pw<NB>()) {
        tile_norms<NB, S>(c, k, k + 1 + (int)blockIdx.x - qr_pw<NB>(), (double *)smem);
        return;
    }
    QrChain ch;  // the GEQRT unit of tile k alone
    ch.top = k; ch.mfirst = k + 1; ch.end = k + 1; ch.epoch = qr_epoch(k, 0);
    ch.geqrt = true; ch.tt = false;
    qr_producer<NB, P64, false, false>(c, k, ch, (int)blockIdx.x, smem, false, c.W + (size_t)k * NB * NB,
                                       c.Dinv + (size_t)k * NB * NB);
}

// QR step k of the flat tree (launch d = 0) with the GEPP of step k+1's
// diagonal tile (GETRF on its FP64 copy, the LU attempt of the next panel) as
// its last workgroup.  That tile is final once the consumers of tile column
// k+1 have applied tile k+1's reflectors (two of the step's sequential
// units), so the GEPP runs beside the rest of the step instead of after it.
// It waits for their counts in eflag[k]; every other workgroup waits only on
// lower-numbered ones, and this one is numbered last, so dispatch order still
// guarantees progress.  Its LDS is the larger of the two routines'.
template <int NB, int P> constexpr int qr_ep_lds() {
    return qr_step_lds<NB, P>() > (int)sizeof(GetrfSmem<NB, 1>) ? qr_step_lds<NB, P>() : (int)sizeof(GetrfSmem<NB, 1>);
}
template <int NB, int P> constexpr int qr_ep_occ() { return qr_ep_lds<NB, P>() <= 80 * 1024 ? 2 : 1; }

template <int NB, int P>
__global__ __launch_bounds__(WG, (qr_ep_occ<NB, P>())) void k_qr_step_ep(Ctx c, int k, int mode) {
    static_assert(NB <= 256, "the tile variant of the GEPP");
    if (c.dec[k] != 0) return;
    __shared__ __attribute__((aligned(16))) char smem[qr_ep_lds<NB, P>()];
    if (blockIdx.x + 1 < gridDim.x) {
        qr_step_body<NB, P, false>(c, k, mode, 0, 1, smem);
        return;
    }
    __shared__ int ready;
    if (threadIdx.x == 0) ready = flag_wait(&c.eflag[k], qr_spc<NB>(), &c.st->watchdog);
    __syncthreads();
    if (!ready) return;
    fence_acquire();
    getrf_core<NB, typename Tr<P>::S, 1>(c, k + 1, smem);
}

// Lookahead resources owned by a factorization handle: two more streams (default
// priority; st for the LU update, st2 for a QR step's R^-1 and T) and the
// events that order them against the caller's stream.
struct Side {
    hipStream_t st, st2;
    hipEvent_t ea, eb, el;
};

struct Ops {
    void (*factor)(const Ctx &, const Layout &, const double *A, int64_t lda, const luqr_opts &, int nsteps,
                   hipStream_t, hipEvent_t *ev, const Side *side);
    void (*solve)(const Ctx &, const Layout &, SolveArgs, const int *hdec, hipStream_t);
    void (*export_factors)(const Ctx &, const Layout &, double *F, int64_t ldf, hipStream_t);
};

inline unsigned nblk(int64_t count, int per = WG) { return (unsigned)((count + per - 1) / per); }

template <int NB, int P>
struct Eng {
    typedef typename Tr<P>::S S;

    // ev (optional): LUQR_NPHASE + 1 events per step, one before each phase of
    // luqr_get_step_times and one after the last.
    // side (optional): lookahead.  Step k's bulk trailing work -- the LU update
    // of columns k+2.. or the QR step's R^-1, Gram and full T -- goes to
    // side->st once step k's critical part (LU: Eliminate/Apply and the update
    // of column k+1; QR: the QR step) is done (event ea), so that step k+1's
    // panel factor, norms and decision run meanwhile on st; step k+1's branch
    // kernels wait for the LU update (event el), while a QR step's R^-1 and
    // full T, which read only tile column k and write only its own buffers,
    // may still run on side->st2 (the factorization ends by waiting for all
    // of it, event eb).  The panel of step k+1 reads only tile column k+1, which the
    // critical part has finished, and writes only its own per-step buffers.
    // Early GEPP (flat tree, variant A1, step k+1 without a domain, nb <=
    // 256): the QR step runs as k_qr_step_ep, and step k+1's panel launch
    // leaves the GEPP out when step k was a QR step.
    static void factor(const Ctx &c, const Layout &L, const double *A, int64_t lda, const luqr_opts &o, int nsteps,
                       hipStream_t st, hipEvent_t *ev, const Side *side) {
        const int n = (int)c.n;
        k_status_reset<<<1, 64, 0, st>>>(c.st);
        k_fill_int<<<nblk((int64_t)n * (NB / IB)), WG, 0, st>>>(c.flags, (int64_t)n * (NB / IB), 0);
        k_fill_int<<<nblk(n), WG, 0, st>>>(c.eflag, n, 0);
        k_fill_int<<<nblk(n), WG, 0, st>>>(c.dec, n, -1);
        k_fill_u32<<<nblk((int64_t)n * n), WG, 0, st>>>(c.tmax, (int64_t)n * n);
        k_to_tiles<S><<<(unsigned)(c.n * c.n), WG, 0, st>>>(A, lda, c.N, c.n, NB, (S *)c.At);
        constexpr int B = NB < 64 ? NB : 64;
        constexpr int E = LUQR_NPHASE + 1;
        auto early_ok = [&](int k) {  // step k's GEPP may run inside QR step k-1
            return NB <= 256 && k > 0 && k < nsteps && !c.a2 && c.qtree == 0 && c.dcount(k) == 1;
        };
        for (int k = 0; k < nsteps; ++k) {
            const int rest = n - k - 1;
            const int pe = early_ok(k) ? 1 : 0;
            if (ev) (void)hipEventRecord(ev[E * k + 0], st);
            // the tile norms of the criterion run as extra workgroups of the
            // launch that factors the diagonal tile
            if (c.a2) {
                // variant A2: GEQRT of A_kk (FP64, on a working copy), Q^T, the
                // rounded factors into the tile, R^{-1}
                k_a2_copy<NB, S><<<NB * NB / (4 * WG), WG, 0, st>>>(c, k);
                k_a2_geqrt<NB, S><<<qr_pw<NB>() + rest, WG, 0, st>>>(c, k);
                k_a2_qt<NB><<<NB / 16, WG, 0, st>>>(c, k);
                k_a2_commit<NB, S><<<NB * NB / (4 * WG), WG, 0, st>>>(c, k);
                k_a2_rinv<NB><<<NB / 4, WG, 0, st>>>(c, k);
            } else {
                if constexpr (NB <= 256) {
                    if (c.dcount(k) > 1) k_panel_getrf<NB, S, 2><<<1 + rest, WG, 0, st>>>(c, k, 0);  // up to 512 stacked rows
                    else k_panel_getrf<NB, S, 1><<<1 + rest, WG, 0, st>>>(c, k, pe);
                } else {
                    k_panel_getrf<NB, S, 2><<<1 + rest, WG, 0, st>>>(c, k, 0);
                }
                k_panel_trtri<NB, S><<<NB / 2 + (pe ? rest : 0), WG, 0, st>>>(c, k, pe);
            }
            if (o.invnorm_estimate) k_panel_invest<NB><<<1, WG, 0, st>>>(c, k);
            else k_panel_invnorm<NB><<<(NB / B) * (NB / B), WG, 0, st>>>(c, k);
            DecideArgs a;
            a.crit = o.criterion;
            a.alpha = o.alpha;
            a.forced_k = (o.criterion == LUQR_CRIT_FORCED) ? o.forced[k] : 0;
            a.seed = o.seed;
            k_panel_decide<NB><<<1, WG, 0, st>>>(c, k, a);
            if (ev) (void)hipEventRecord(ev[E * k + 1], st);
            if (side && k > 0) (void)hipStreamWaitEvent(st, side->el, 0);  // step k-1's LU update
            if (c.dcount(k) > 1) k_domain_swap<NB, P><<<(unsigned)rest * (NB / DSW_CW), WG, 0, st>>>(c, k);
            k_lu_apply<NB, P><<<1 + 2 * rest * (NB / lu_rb<NB>()), WG, 0, st>>>(c, k);
            if (ev) (void)hipEventRecord(ev[E * k + 2], st);
            constexpr int PER = NB / upd_bt<NB>();
            if (rest > 0) {  // with lookahead column k+1 only, the rest below
                const unsigned cols = side ? 1u : (unsigned)rest;
                k_lu_update<NB, P><<<(unsigned)rest * cols * PER * PER, WG, 0, st>>>(c, k, k + 1);
            }
            if (ev) (void)hipEventRecord(ev[E * k + 3], st);
            {  // the groups' chains, then the TT levels of the elimination tree
                const QrTree tr(n, k, c.qtree);
                const int mode = c.a2 ? QR_REST : QR_FULL;
                const unsigned per = qr_pw<NB>() + rest * qr_spc<NB>();
                const unsigned grid = tr.G * per + qr_keepers<NB, P>(n, k, tr.G);
                if constexpr (NB <= 256) {
                    if (early_ok(k + 1)) k_qr_step_ep<NB, P><<<grid + 1, WG, 0, st>>>(c, k, mode);
                    else k_qr_step<NB, P, false><<<grid, WG, 0, st>>>(c, k, mode, 0);
                } else {
                    k_qr_step<NB, P, false><<<grid, WG, 0, st>>>(c, k, mode, 0);
                }
                for (int d = 1; d < tr.G; d *= 2)
                    k_qr_step<NB, P, true><<<tr.npairs(d) * per, WG, 0, st>>>(c, k, mode, d);
            }
            if (ev) (void)hipEventRecord(ev[E * k + 4], st);
            hipStream_t sb = st;
            if (side) {
                (void)hipEventRecord(side->ea, st);
                (void)hipStreamWaitEvent(side->st, side->ea, 0);
                if (rest > 1)
                    k_lu_update<NB, P><<<(unsigned)rest * (rest - 1) * PER * PER, WG, 0, side->st>>>(c, k, k + 2);
                (void)hipEventRecord(side->el, side->st);
                // a QR step's R^-1 and T completion on a third stream, so that
                // the next LU step's update is not queued behind them
                (void)hipStreamWaitEvent(side->st2, side->ea, 0);
                sb = side->st2;
            }
            // QR steps: R_kk after every TSQRT (A2's panel inverted the GEQRT's R for the criterion)
            k_qr_rinv<NB, S><<<NB / 4, WG, 0, sb>>>(c, k);
            if constexpr (NB > IB) {
                k_qr_gram<NB, P><<<dim3(qr_npairs<NB>(), n - k), WG, 0, sb>>>(c, k, 0);
                k_qr_tfull<NB, P><<<n - k, WG, 0, sb>>>(c, k, 0);
                if (c.qtree > 0 && QrTree(n, k, c.qtree).G > 1) {  // the TT factors of the killed heads
                    k_qr_gram<NB, P><<<dim3(qr_npairs<NB>(), n - k), WG, 0, sb>>>(c, k, 1);
                    k_qr_tfull<NB, P><<<n - k, WG, 0, sb>>>(c, k, 1);
                }
            }
            if (side) {  // eb: all of step k's bulk work, the LU update included
                (void)hipStreamWaitEvent(sb, side->el, 0);
                (void)hipEventRecord(side->eb, sb);
            }
            if (ev) (void)hipEventRecord(ev[E * k + 5], sb);
        }
        if (side) (void)hipStreamWaitEvent(st, side->eb, 0);  // join: the factorization ends on st
    }

    // hdec: the decision sequence on the host, if the caller has it: only the
    // chosen branch of each step is launched.  nullptr: both branches are
    // launched and the kernels of the other one return at once (they read the
    // decision on the device), so the solve needs no host round trip.
    static void solve(const Ctx &c, const Layout &L, SolveArgs s, const int *hdec, hipStream_t st) {
        const int n = (int)c.n;
        const unsigned ch = (unsigned)((s.nrhs + rq<NB>() - 1) / rq<NB>());
        constexpr int RPT = NB / mv_rb<NB>();  // row blocks per tile
        bool wave = false;
        if constexpr (NB == 256 && sizeof(S) == 4) {
            // the forward pass as one wavefront launch; the tile counters reuse
            // the QR steps' flags (n * nb/IB ints, free once the factorization is done)
            const int wch = (s.nrhs + FW_RQ - 1) / FW_RQ;
            if (c.dstride == 0 && c.qtree == 0 && wch <= 4) {  // its QR rows follow the flat tree
                k_fill_int<<<nblk((int64_t)n * wch), WG, 0, st>>>(c.flags, (int64_t)n * wch, 0);
                k_fwd_wave<NB, S><<<dim3(n, wch), FW_WG, 0, st>>>(c, s, c.flags);
                wave = true;
            }
        }
        for (int k = 0; k < n && !wave; ++k) {
            const int rest = n - k - 1;
            if (!hdec || hdec[k] == 1) {
                if (c.dcount(k) > 1) k_fwd_dswap<NB><<<dim3(1, (unsigned)((s.nrhs + 15) / 16)), WG, 0, st>>>(c, s, k);
                k_fwd_lu_a<NB><<<dim3(RPT, ch), WG, 0, st>>>(c, s, k);
                if (rest > 0) k_fwd_lu_b<NB, S><<<dim3(rest * RPT, ch), WG, 0, st>>>(c, s, k);
            }
            if (!hdec || hdec[k] == 0) {
                const QrTree tr(n, k, c.qtree);
                if (rest > 0) k_fwd_qr_g<NB, S><<<dim3(rest * qs<NB>(), ch), WG, 0, st>>>(c, s, k);
                k_fwd_qr_chain<NB, S><<<dim3(tr.G, ch), chain_wg<NB, S>(), 0, st>>>(c, s, k);
                if (rest > 0) k_fwd_qr_u<NB, S><<<dim3(rest * RPT, ch), WG, 0, st>>>(c, s, k);
                if (c.qtree > 0) {
                    for (int d = 1; d < tr.G; d *= 2) k_fwd_tt<NB, S><<<dim3(tr.npairs(d), ch), WG, 0, st>>>(c, s, k, d);
                    k_fwd_tt_fin<NB><<<nblk((int64_t)NB * s.nrhs), WG, 0, st>>>(c, s, k);
                }
            }
        }
        bool bwave = false;
        if constexpr (NB == 256 && sizeof(S) == 4) {
            // the back substitution as one wavefront launch; its counters follow
            // the forward pass's in the QR steps' flags (n * nb/IB ints)
            const int wch = (s.nrhs + FW_RQ - 1) / FW_RQ;
            if (wch <= 4) {
                int *cb = c.flags + (size_t)n * 4;
                k_fill_int<<<nblk((int64_t)n * wch), WG, 0, st>>>(cb, (int64_t)n * wch, 0);
                k_bwd_wave<NB, S><<<dim3(n, wch), FW_WG, 0, st>>>(c, s, cb);
                bwave = true;
            }
        }
        for (int k = n - 1; k >= 0 && !bwave; --k) {
            k_bwd_a<NB><<<dim3(RPT, ch), WG, 0, st>>>(c, s, k);
            if (k > 0) k_bwd_b<NB, S><<<dim3(k * RPT, ch), WG, 0, st>>>(c, s, k);
        }
    }

    static void export_factors(const Ctx &c, const Layout &L, double *F, int64_t ldf, hipStream_t st) {
        k_from_tiles<S><<<nblk(c.N * c.N), WG, 0, st>>>((const S *)c.At, c.n, NB, c.N, F, ldf);
    }

    static const Ops *ops() {
        static const Ops o = {&factor, &solve, &export_factors};
        return &o;
    }
};

// Launch tables, one per (tile size, precision) instantiation (inst.hip).
template <int NB, int P> const Ops *eng_ops();
#define LQ_DECLARE(NB, P) template <> const Ops *eng_ops<NB, P>();
LQ_DECLARE(32, P64) LQ_DECLARE(64, P64) LQ_DECLARE(128, P64) LQ_DECLARE(256, P64)
LQ_DECLARE(32, P32) LQ_DECLARE(64, P32) LQ_DECLARE(128, P32) LQ_DECLARE(256, P32) LQ_DECLARE(512, P32)
LQ_DECLARE(32, PB16) LQ_DECLARE(64, PB16) LQ_DECLARE(128, PB16) LQ_DECLARE(256, PB16) LQ_DECLARE(512, PB16)
#undef LQ_DECLARE

template <int P> const Ops *ops_nb(int nb) {
    switch (nb) {
    case 32: return eng_ops<32, P>();
    case 64: return eng_ops<64, P>();
    case 128: return eng_ops<128, P>();
    case 256: return eng_ops<256, P>();
    case 512: if constexpr (P != P64) return eng_ops<512, P>(); else return nullptr;
    default: return nullptr;
    }
}

}  // namespace lq
