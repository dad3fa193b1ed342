// solver.hip -- conjugate gradient on M^dag M (eq. 3-4: the inverse of the
// two-flavour fermion matrix applied to the pseudofermion), batched over
// right-hand sides, in FP64 or mixed precision with FP64 reliable updates.
//
// Even-odd iteration (A = Mhat^dag Mhat, Mhat = 1 - kappa^2 D_eo D_oe), per
// active RHS, four stencil sweeps and one vector kernel:
//   t_o  = D_oe p                                   (sweep 1)
//   t2   = p - k^2 D_eo t_o,  pAp = |t2|^2           (sweep 2, fused norm)
//   alpha = rr / pAp                                 (finalize, on device)
//   t_o  = D_oe^dag t2                               (sweep 3)
//   Ap   = t2 - k^2 D_eo^dag t_o;  x += alpha p;  r -= alpha Ap;  rr' = |r|^2
//                                                    (sweep 4, fused update)
//   beta = rr' / rr                                  (finalize, on device)
//   p    = r + beta p
// alpha and beta never leave the device; the host reads the residual norms
// every `poll` iterations.  In mixed precision p, r and the intermediates are
// FP32 or FP16 (per-site norm) and the solution increment accumulates in
// FP32; when |r| falls below delta * (its maximum since the last update), or
// the sloppy residual claims convergence, the FP64 solution is advanced and
// the residual is recomputed as b - A x in FP64 (reliable update).
// Convergence is declared only on that FP64 true residual.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "wd_internal.h"

namespace wd {

namespace {

struct Scalars {
    double *bb, *rr, *alpha, *beta, *coef1, *coef2, *partial;
    int pstride;
};

struct Ops {
    wd_ctx *c;
    int eo;
    Scalars s;
    const TuneCfg *cfg;
};

// out = A in for the active RHS in precision (sp, lk), using t_o / t_e as
// temporaries (eo) or T (full).  When pAp != nullptr the first half's norm
// partials go to the scalar partial buffer (pAp = |M in|^2).
wd_status apply_A(const Ops &o, int sp, int lk, const Field &in, const Field &out,
                  const Field &t_o, const Field &t_e, const int *act, int nact, bool norm)
{
    wd_ctx *c = o.c;
    Sweep sw;
    sw.sp = sp;
    sw.lk = lk;
    sw.xp = sp;
    sw.active = act;
    sw.nact = nact;
    if (o.eo) {
        sw.coef = o.s.coef2;
        sw.P = 1; sw.dag = 0; sw.epi = EPI_PLAIN; sw.in = in; sw.out = t_o;
        WD_TRY(run_sweep(c, sw, o.cfg));
        sw.P = 0; sw.epi = EPI_XPAY; sw.in = t_o; sw.x = in; sw.out = t_e;
        sw.partial = norm ? o.s.partial : nullptr; sw.pstride = o.s.pstride; sw.pw_off = 0;
        WD_TRY(run_sweep(c, sw, o.cfg));
        sw.partial = nullptr;
        sw.P = 1; sw.dag = 1; sw.epi = EPI_PLAIN; sw.in = t_e; sw.out = t_o;
        WD_TRY(run_sweep(c, sw, o.cfg));
        sw.P = 0; sw.epi = EPI_XPAY; sw.in = t_o; sw.x = t_e; sw.out = out;
        WD_TRY(run_sweep(c, sw, o.cfg));
    } else {
        // T = M in (both parities), out = M^dag T
        const Field &T = t_e;
        sw.coef = o.s.coef1;
        sw.epi = EPI_XPAY;
        for (int pass = 0; pass < 2; pass++) {
            const Field &src = pass ? T : in;
            const Field &dst = pass ? out : T;
            sw.dag = pass;
            for (int P = 0; P < 2; P++) {
                sw.P = P;
                sw.in = sub_view(src, 1 - P);
                sw.x = sub_view(src, P);
                sw.out = sub_view(dst, P);
                sw.partial = (norm && pass == 0) ? o.s.partial : nullptr;
                sw.pstride = o.s.pstride;
                sw.pw_off = P * ngroups_of((int)c->Vh);
                WD_TRY(run_sweep(c, sw, o.cfg));
            }
        }
    }
    return WD_OK;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                          \
        hipError_t e__ = (expr);                                                                  \
        if (e__ != hipSuccess)                                                                    \
            return set_error(WD_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__, __LINE__); \
    } while (0)

}  // namespace

}  // namespace wd

using namespace wd;

extern "C" wd_status wd_cg_solve(wd_ctx *c, double *x, const double *phi, int nrhs,
                                 const double *kappa, const wd_solver_params *pin,
                                 wd_solver_stats *st)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !x || !phi || !kappa) return set_error(WD_ERR_ARG, "NULL argument");
    if (nrhs < 1) return set_error(WD_ERR_ARG, "nrhs = %d", nrhs);
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    wd_solver_params p;
    wd_solver_defaults(&p);
    if (pin) p = *pin;
    if (!(p.tol > 0) || p.maxiter < 0 || p.poll < 1 || !(p.delta > 0 && p.delta < 1))
        return set_error(WD_ERR_ARG, "bad solver parameters (tol %g maxiter %d poll %d delta %g)",
                         p.tol, p.maxiter, p.poll, p.delta);
    int sp, lk, xp;
    WD_TRY(decode_prec(c, p.prec_sloppy, &sp, &lk, &xp));
    if (!p.eo && sp != SP_F64)
        return set_error(WD_ERR_ARG, "the full-lattice solver runs in FP64 only");
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(kappa[j])) return set_error(WD_ERR_ARG, "kappa[%d] not finite", j);
    WD_HIP(hipSetDevice(c->device));

    const bool mixed = sp != SP_F64;
    const int nsub = p.eo ? 1 : 2;
    const int Vh = (int)c->Vh;
    const hipStream_t s = c->stream;

    // scalars: bb, rr, alpha, beta, coef1, coef2 (nrhs each) + partials
    const int nw1 = ngroups_of(Vh);
    const int pstride = 2 * nw1 + 1;
    std::vector<double> hc1(nrhs), hc2(nrhs);
    for (int j = 0; j < nrhs; j++) {
        hc1[j] = -kappa[j];
        hc2[j] = -kappa[j] * kappa[j];
    }
    Scalars sc;
    void *vp;
    WD_TRY(ws_get(c, "cg_scal", sizeof(double) * 6 * nrhs, &vp));
    sc.bb = (double *)vp;
    sc.rr = sc.bb + nrhs;
    sc.alpha = sc.rr + nrhs;
    sc.beta = sc.alpha + nrhs;
    double *dre = sc.beta + nrhs, *dim = dre + nrhs;  // <r, p> after a reliable update
    WD_TRY(upload_doubles(c, "cg_coef1", hc1.data(), nrhs, &sc.coef1));
    WD_TRY(upload_doubles(c, "cg_coef2", hc2.data(), nrhs, &sc.coef2));
    WD_TRY(ws_get(c, "cg_partial", sizeof(double) * pstride * nrhs * 2, &vp));
    sc.partial = (double *)vp;
    double *partial2 = sc.partial + (size_t)pstride * nrhs;
    sc.pstride = pstride;
    const TuneCfg *cfg = nullptr;  // per-sweep shapes come from the tuner when p.tuned
    Ops o{c, p.eo, sc, cfg};
    struct TunedScope {
        wd_ctx *c;
        bool old;
        ~TunedScope() { c->use_tuned = old; }
    } tscope{c, c->use_tuned};
    c->use_tuned = p.tuned != 0;

    // fields
    Field b64, x64, r64, to64, te64, Ap64;
    WD_TRY(alloc_field(c, "cg_b", SP_F64, nsub, nrhs, &b64));
    WD_TRY(alloc_field(c, "cg_x", SP_F64, nsub, nrhs, &x64));
    WD_TRY(alloc_field(c, "cg_r", SP_F64, nsub, nrhs, &r64));
    WD_TRY(alloc_field(c, "cg_to", SP_F64, 1, nrhs, &to64));
    WD_TRY(alloc_field(c, "cg_te", SP_F64, nsub, nrhs, &te64));
    WD_TRY(alloc_field(c, "cg_ap", SP_F64, nsub, nrhs, &Ap64));
    Field ps, rs, t2s, tos, xs;
    if (mixed) {
        WD_TRY(alloc_field(c, "cg_ps", sp, 1, nrhs, &ps));
        WD_TRY(alloc_field(c, "cg_rs", sp, 1, nrhs, &rs));
        WD_TRY(alloc_field(c, "cg_t2s", sp, 1, nrhs, &t2s));
        WD_TRY(alloc_field(c, "cg_tos", sp, 1, nrhs, &tos));
        WD_TRY(alloc_field(c, "cg_xs", xp, 1, nrhs, &xs));
    } else {
        WD_TRY(alloc_field(c, "cg_p", SP_F64, nsub, nrhs, &ps));
        rs = r64;
        t2s = te64;
        tos = to64;
        xs = x64;
    }

    // all RHS ids
    std::vector<int> all(nrhs);
    for (int j = 0; j < nrhs; j++) all[j] = j;
    int *act_all, *act, *act_ru;
    WD_TRY(upload_ints(c, "cg_act_all", all.data(), nrhs, &act_all));

    hipError_t e;
    if ((e = pack_spinor(phi, b64, nrhs, p.eo ? 0 : 1, c->g, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
    const int nwF = p.eo ? nw1 : ngroups_of(2 * Vh);  // BLAS partial count
    const int nwD = p.eo ? nw1 : 2 * nw1;            // stencil partial count
    HIPCHK(blas_norm(b64, Vh, act_all, nrhs, sc.partial, pstride, s));
    HIPCHK(blas_finalize(sc.partial, pstride, nwF, act_all, nrhs, FIN_STORE, sc.rr, sc.alpha, sc.beta, sc.bb, s));
    HIPCHK(hipMemcpyAsync(sc.rr, sc.bb, sizeof(double) * nrhs, hipMemcpyDeviceToDevice, s));
    HIPCHK(blas_zero(x64, Vh, act_all, nrhs, s));
    HIPCHK(blas_copy(r64, b64, Vh, act_all, nrhs, s));
    if (mixed) {
        HIPCHK(blas_copy(rs, b64, Vh, act_all, nrhs, s));
        HIPCHK(blas_zero(xs, Vh, act_all, nrhs, s));
    }
    HIPCHK(blas_copy(ps, rs, Vh, act_all, nrhs, s));

    double *hbuf;
    WD_TRY(pinned_get(c, 1, sizeof(double) * nrhs, &vp));
    hbuf = (double *)vp;
    HIPCHK(hipMemcpyAsync(hbuf, sc.bb, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<double> bb(hbuf, hbuf + nrhs), maxrr(nrhs), rrh(nrhs), prevtrue(hbuf, hbuf + nrhs);
    std::vector<int> restart;
    std::vector<int> iters(nrhs, 0), rus(nrhs, 0), status(nrhs, WD_ERR_NOCONV);
    std::vector<double> tres(nrhs, 0.0);
    std::vector<int> active;
    for (int j = 0; j < nrhs; j++) {
        if (!std::isfinite(bb[j])) {
            status[j] = WD_ERR_NAN;
            tres[j] = NAN;
        } else if (bb[j] == 0.0) {
            status[j] = WD_OK;
        } else {
            active.push_back(j);
            maxrr[j] = bb[j];
        }
    }
    const double tol2 = p.tol * p.tol, d2 = p.delta * p.delta;
    // WD_SOLVER_TRACE=1 prints the residual history to stderr (diagnostics)
    const char *trace_env = getenv("WD_SOLVER_TRACE");
    const bool trace = trace_env && trace_env[0] == '1';

    auto upload_active = [&](const std::vector<int> &v, const char *name, int **dev) -> wd_status {
        return upload_ints(c, name, v.data(), (int)v.size(), dev);
    };
    WD_TRY(upload_active(active, "cg_act", &act));

    // reliable update of the listed RHS: x64 += xs, r64 = b - A x64 (FP64),
    // rr = |r64|^2, rs = r64.  The search direction p = r + beta p_old was
    // built from the replaced residual; it is rebuilt as r_new + q with
    // q = p - r_old = beta p_old made orthogonal to r_new
    // (q -= <r_new, q> / <r_new, r_new> r_new).  Returns the new rr in rrh.
    auto reliable = [&](const std::vector<int> &ids) -> wd_status {
        if (ids.empty()) return WD_OK;
        WD_TRY(upload_active(ids, "cg_act_ru", &act_ru));
        const int n = (int)ids.size();
        HIPCHK(blas_axpy_const(ps, rs, -1.0, Vh, act_ru, n, s));
        if (mixed) HIPCHK(blas_add_zero(x64, xs, Vh, act_ru, n, s));
        WD_TRY(apply_A(o, SP_F64, c->lk64, x64, Ap64, to64, te64, act_ru, n, false));
        HIPCHK(blas_resid(r64, b64, Ap64, Vh, act_ru, n, sc.partial, pstride, s));
        HIPCHK(blas_finalize(sc.partial, pstride, nwF, act_ru, n, FIN_RR, sc.rr, sc.alpha, sc.beta, nullptr, s));
        if (mixed) HIPCHK(blas_copy(rs, r64, Vh, act_ru, n, s));
        HIPCHK(blas_cdot(rs, ps, Vh, act_ru, n, sc.partial, partial2, pstride, s));
        HIPCHK(blas_finalize(sc.partial, pstride, nwF, act_ru, n, FIN_STORE, sc.rr, sc.alpha, sc.beta, dre, s));
        HIPCHK(blas_finalize(partial2, pstride, nwF, act_ru, n, FIN_STORE, sc.rr, sc.alpha, sc.beta, dim, s));
        HIPCHK(blas_orth(ps, rs, dre, dim, sc.rr, Vh, act_ru, n, s));
        HIPCHK(blas_axpy_const(ps, rs, 1.0, Vh, act_ru, n, s));
        HIPCHK(hipMemcpyAsync(hbuf, sc.rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int j : ids) rrh[j] = hbuf[j];
        return WD_OK;
    };

    int it = 0;
    while (!active.empty() && it < p.maxiter) {
        const int nact = (int)active.size();
        const int k = std::min(p.poll, p.maxiter - it);
        for (int kk = 0; kk < k; kk++) {
            Sweep sw;
            sw.sp = sp; sw.lk = lk; sw.xp = xp; sw.active = act; sw.nact = nact;
            if (p.eo) {
                sw.coef = sc.coef2;
                sw.P = 1; sw.dag = 0; sw.epi = EPI_PLAIN; sw.in = ps; sw.out = tos;
                WD_TRY(run_sweep(c, sw, cfg));
                sw.P = 0; sw.epi = EPI_XPAY; sw.in = tos; sw.x = ps; sw.out = t2s;
                sw.partial = sc.partial; sw.pstride = pstride; sw.pw_off = 0;
                WD_TRY(run_sweep(c, sw, cfg));
                HIPCHK(blas_finalize(sc.partial, pstride, nwD, act, nact, FIN_ALPHA, sc.rr, sc.alpha, sc.beta, nullptr, s));
                sw.partial = nullptr;
                sw.P = 1; sw.dag = 1; sw.epi = EPI_PLAIN; sw.in = t2s; sw.out = tos;
                WD_TRY(run_sweep(c, sw, cfg));
                sw.P = 0; sw.epi = EPI_CGUPD; sw.in = tos; sw.x = t2s; sw.p = ps; sw.xs = xs; sw.r = rs;
                sw.alpha = sc.alpha; sw.partial = sc.partial;
                WD_TRY(run_sweep(c, sw, cfg));
                HIPCHK(blas_finalize(sc.partial, pstride, nw1, act, nact, FIN_BETA, sc.rr, sc.alpha, sc.beta, nullptr, s));
            } else {
                WD_TRY(apply_A(o, sp, lk, ps, Ap64, to64, te64, act, nact, true));
                HIPCHK(blas_finalize(sc.partial, pstride, nwD, act, nact, FIN_ALPHA, sc.rr, sc.alpha, sc.beta, nullptr, s));
                HIPCHK(blas_cg_update(xs, ps, rs, Ap64, sc.alpha, Vh, act, nact, sc.partial, pstride, s));
                HIPCHK(blas_finalize(sc.partial, pstride, nwF, act, nact, FIN_BETA, sc.rr, sc.alpha, sc.beta, nullptr, s));
            }
            HIPCHK(blas_p_update(ps, rs, sc.beta, Vh, act, nact, s));
        }
        it += k;
        for (int j : active) iters[j] = it;
        HIPCHK(hipMemcpyAsync(hbuf, sc.rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int> ru, keep;
        if (trace)
            for (int j : active) fprintf(stderr, "[wd cg] it %d rhs %d sloppy |r|/|b| %.3e\n", it, j, std::sqrt(hbuf[j] / bb[j]));
        for (int j : active) {
            const double r2 = hbuf[j];
            if (!std::isfinite(r2)) {
                status[j] = WD_ERR_NAN;
                continue;
            }
            if (r2 <= tol2 * bb[j] || (mixed && r2 < d2 * maxrr[j])) ru.push_back(j);
            if (r2 > maxrr[j]) maxrr[j] = r2;
            keep.push_back(j);
        }
        if (!ru.empty()) {
            WD_TRY(reliable(ru));
            std::vector<int> keep2;
            for (int j : keep) {
                bool done = false;
                for (int q : ru)
                    if (q == j) {
                        rus[j]++;
                        if (trace) fprintf(stderr, "[wd cg] it %d rhs %d reliable update: true |r|/|b| %.3e\n", it, j, std::sqrt(rrh[j] / bb[j]));
                        if (!std::isfinite(rrh[j])) {
                            status[j] = WD_ERR_NAN;
                            done = true;
                        } else if (rrh[j] <= tol2 * bb[j]) {
                            status[j] = WD_OK;
                            tres[j] = std::sqrt(rrh[j] / bb[j]);
                            done = true;
                        } else {
                            maxrr[j] = rrh[j];
                            // a replacement that did not halve the true residual
                            // means the sloppy iteration has stalled: restart
                            if (rrh[j] > 0.25 * prevtrue[j]) restart.push_back(j);
                            prevtrue[j] = rrh[j];
                        }
                    }
                if (!done) keep2.push_back(j);
            }
            keep.swap(keep2);
            if (!restart.empty()) {
                int *act_rs;
                WD_TRY(upload_active(restart, "cg_act_rs", &act_rs));
                HIPCHK(blas_copy(ps, rs, Vh, act_rs, (int)restart.size(), s));
                if (trace)
                    for (int j : restart) fprintf(stderr, "[wd cg] it %d rhs %d restart p = r\n", it, j);
                restart.clear();
            }
        }
        if (keep.size() != active.size()) {
            active.swap(keep);
            WD_TRY(upload_active(active, "cg_act", &act));
        }
    }
    // unconverged RHS: fold in the sloppy increment and report the true residual
    if (!active.empty()) {
        WD_TRY(reliable(active));
        for (int j : active) {
            rus[j]++;
            tres[j] = std::sqrt(rrh[j] / bb[j]);
            status[j] = std::isfinite(rrh[j]) ? WD_ERR_NOCONV : WD_ERR_NAN;
        }
    }
    if ((e = unpack_spinor(x64, x, nrhs, p.eo ? 0 : 1, c->g, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    wd_status ret = WD_OK;
    for (int j = 0; j < nrhs; j++) {
        if (st) {
            st[j].iters = iters[j];
            st[j].reliable_updates = rus[j];
            st[j].true_resid = tres[j];
            st[j].seconds = secs;
            st[j].status = status[j];
        }
        if (status[j] == WD_ERR_NAN) ret = WD_ERR_NAN;
        else if (status[j] != WD_OK && ret == WD_OK) ret = (wd_status)status[j];
    }
    if (ret != WD_OK) set_error(ret, "%s", ret == WD_ERR_NAN ? "non-finite residual" : "not converged");
    return ret;
}
