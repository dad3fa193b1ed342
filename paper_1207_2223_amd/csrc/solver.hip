// solver.hip -- conjugate gradient on M^dag M (eq. 3-4: the inverse of the
// two-flavour fermion matrix applied to the pseudofermion), batched over
// right-hand sides, in FP64 or mixed precision with FP64 reliable updates,
// and persistent solver sessions for continuous batching.
//
// Even-odd iteration (A = Mhat^dag Mhat, Mhat = 1 - kappa^2 D_eo D_oe), per
// active RHS, four stencil sweeps and one vector kernel:
//   t_o  = D_oe p                                   (sweep 1)
//   t2   = p - k^2 D_eo t_o,  pAp = |t2|^2           (sweep 2, fused norm)
//   t_o  = D_oe^dag t2                               (sweep 3; its leading
//   alpha = rr / pAp                                  work-groups finalize alpha)
//   Ap   = t2 - k^2 D_eo^dag t_o;  r -= alpha Ap;  rr' = |r|^2
//                                                    (sweep 4, fused update)
//   beta = rr' / rr                                  (finalize, on device)
//   p'   = r + beta p
// alpha and beta never leave the device; the host reads the residual norms
// after every step of k iterations.  The solution is not touched by the
// iteration itself: each iteration's p goes to its own slot of a ring of
// kRing directions (and alpha to a matching history; in a mixed solve -- an
// FP64 solve keeps a ring of one), and every kRing
// iterations, and at the end of each step, the p update first adds
// alpha_j p_j of the iterations since the last flush to x, in iteration
// order -- the same roundings as x += alpha p once per iteration, with the
// solution read and written once per flush instead of once per iteration.  In mixed precision p, r and the
// intermediates are FP32 or FP16 (per-site norm) and the solution increment
// accumulates in FP32; when |r| falls below delta * (its maximum since the
// last update), or the sloppy residual claims convergence, the FP64 solution
// is advanced and the residual is recomputed as b - A x in FP64 (reliable
// update).  Convergence is declared only on that FP64 true residual.
//
// Every decision for a right-hand side depends only on its own residual
// history at multiples of k of its own iteration count, and the kernels treat
// every RHS independently (fixed reduction trees), so a RHS gives the same
// bits whether it is solved alone or batched with others joining at step
// boundaries.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "wd_internal.h"

namespace wd {

namespace {

#define HIPCHK(expr)                                                                               \
    do {                                                                                          \
        hipError_t e__ = (expr);                                                                  \
        if (e__ != hipSuccess)                                                                    \
            return set_error(WD_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__, __LINE__); \
    } while (0)

enum { SLOT_FREE = 0, SLOT_RUNNING = 1, SLOT_DONE = 2 };

}  // namespace

struct BatchSolver {
    // one set of iterated fields: the sloppy lane (prec_sloppy), or the FP64
    // lane that finishes right-hand sides escalated out of the sloppy one
    struct Lane {
        int sp, lk, xp;
        Field P, R, T2, TO, X;
        bool sloppy;  // X is an increment added to x64 at reliable updates
        std::vector<Field> Pr;  // even-odd: ring of search directions, Pr[0] == P
    };

    // a slot whose FP64 true residual has not reached a new minimum over this
    // many consecutive reliable updates leaves the sloppy lane for FP64
    static constexpr int kStallUpdates = 3;
    // a sloppy slot gets a reliable update at least this often (iterations)
    static constexpr int kMaxItersPerUpdate = 256;
    // restart p = r when the true residual exceeds the recursive one by more
    // than this factor (in |r|^2): the recursion has lost its accuracy
    static constexpr double kDriftRestart = 4.0;
    static constexpr int kScalars = 9;  // per-slot device scalars (bb .. rr_s)
    // directions kept between solution flushes (even-odd lanes; a mixed
    // solve's FP64 lane, used by escalated RHS only, flushes every iteration)
    static constexpr int kRing = kMaxRing;
    static constexpr size_t kMaxGraphs = 32;  // captured steps kept per context

    wd_ctx *c = nullptr;
    wd_solver_params p{};
    std::string pre;  // workspace name prefix
    int cap = 0, sp = 0, lk = 0, xp = 0, nsub = 1, Vh = 0;
    bool mixed = false;
    int pstride = 0, nw1 = 0, nwF = 0, nwD = 0;
    Field b64, x64, r64, to64, te64, Ap64, p64, ps, rs, t2s, tos, xs;
    Lane lane_s{}, lane_d{};
    double *bb = nullptr, *rr = nullptr, *alpha = nullptr, *beta = nullptr, *dre = nullptr, *dim = nullptr;
    double *coef1 = nullptr, *coef2 = nullptr, *partial = nullptr, *partial2 = nullptr;
    double *rr_s = nullptr;  // recursive |r|^2 saved at a reliable update
    double *ahist = nullptr; // alpha of the iterations since the last flush, [kRing][cap]
    double *hbuf = nullptr;  // pinned, cap doubles
    int *act = nullptr, *act64 = nullptr, *lst = nullptr;  // device id lists
    std::vector<int> state, iters, iters64, rus, status, last_ru, stall, active, active64;
    std::vector<double> bbh, maxrr, best, tres, kap;
    bool trace = false;
    bool fold = true;  // alpha finalized inside sweep 3 (else by its own kernel)

    std::string nm(const char *s) const { return pre + s; }
    std::string ring_name(int j) const { return pre + (mixed ? "ps@" : "p@") + std::to_string(j); }

    wd_status init(wd_ctx *ctx, int capacity, const wd_solver_params &prm, const std::string &prefix)
    {
        c = ctx;
        p = prm;
        pre = prefix;
        WD_TRY(decode_prec(c, p.prec_sloppy, &sp, &lk, &xp));
        if (!p.eo && sp != SP_F64) return set_error(WD_ERR_ARG, "the full-lattice solver runs in FP64 only");
        mixed = sp != SP_F64;
        nsub = p.eo ? 1 : 2;
        Vh = (int)c->Vh;
        nw1 = ngroups_of(Vh);
        pstride = 2 * nw1 + 1;
        nwF = p.eo ? nw1 : ngroups_of(2 * Vh);
        nwD = p.eo ? nw1 : 2 * nw1;
        WD_TRY(bind(capacity));
        state.assign(cap, SLOT_FREE);
        iters.assign(cap, 0);
        iters64.assign(cap, 0);
        rus.assign(cap, 0);
        status.assign(cap, WD_OK);
        last_ru.assign(cap, 0);
        stall.assign(cap, 0);
        bbh.assign(cap, 0.0);
        maxrr.assign(cap, 0.0);
        best.assign(cap, 0.0);
        tres.assign(cap, 0.0);
        kap.assign(cap, 0.0);
        active.clear();
        active64.clear();
        const char *te = getenv("WD_SOLVER_TRACE");
        trace = te && te[0] == '1';
        // WD_SEPARATE_FINALIZE=1: alpha by the separate finalize kernel (the
        // same summation order; for checking that both give the same bits)
        const char *sf = getenv("WD_SEPARATE_FINALIZE");
        fold = !(sf && sf[0] == '1');
        return WD_OK;
    }

    // Device state of `capacity` slots (the named workspaces are created, or
    // found with at least the needed size) and the pinned read-back buffer.
    wd_status bind(int capacity)
    {
        cap = capacity;
        void *vp;
        WD_TRY(ws_get(c, nm("scal"), sizeof(double) * kScalars * cap, &vp));
        bb = (double *)vp;
        rr = bb + cap;
        alpha = rr + cap;
        beta = alpha + cap;
        dre = beta + cap;
        dim = dre + cap;
        coef1 = dim + cap;
        coef2 = coef1 + cap;
        rr_s = coef2 + cap;
        WD_TRY(ws_get(c, nm("partial"), sizeof(double) * pstride * cap * 2, &vp));
        partial = (double *)vp;
        partial2 = partial + (size_t)pstride * cap;
        WD_TRY(ws_get(c, nm("ids"), sizeof(int) * 3 * cap, &vp));
        act = (int *)vp;
        act64 = act + cap;
        lst = act64 + cap;
        WD_TRY(ws_get(c, nm("ahist"), sizeof(double) * kRing * cap, &vp));
        ahist = (double *)vp;
        WD_TRY(alloc_field(c, nm("b"), SP_F64, nsub, cap, &b64));
        WD_TRY(alloc_field(c, nm("x"), SP_F64, nsub, cap, &x64));
        WD_TRY(alloc_field(c, nm("r"), SP_F64, nsub, cap, &r64));
        WD_TRY(alloc_field(c, nm("to"), SP_F64, 1, cap, &to64));
        WD_TRY(alloc_field(c, nm("te"), SP_F64, nsub, cap, &te64));
        WD_TRY(alloc_field(c, nm("ap"), SP_F64, nsub, cap, &Ap64));
        WD_TRY(alloc_field(c, nm("p"), SP_F64, nsub, cap, &p64));
        lane_d = Lane{SP_F64, c->lk64, SP_F64, p64, r64, te64, to64, x64, false, {p64}};
        if (mixed) {
            WD_TRY(alloc_field(c, nm("ps"), sp, 1, cap, &ps));
            WD_TRY(alloc_field(c, nm("rs"), sp, 1, cap, &rs));
            WD_TRY(alloc_field(c, nm("t2s"), sp, 1, cap, &t2s));
            WD_TRY(alloc_field(c, nm("tos"), sp, 1, cap, &tos));
            WD_TRY(alloc_field(c, nm("xs"), xp, 1, cap, &xs));
            lane_s = Lane{sp, lk, xp, ps, rs, t2s, tos, xs, true, {ps}};
        }
        // the ring slots 1 .. kRing-1 of the sloppy lane; an FP64 solve keeps
        // a ring of one (x advanced every iteration), which holds its memory
        // per RHS at seven FP64 vectors for serving
        if (p.eo && mixed)
            for (int j = 1; j < kRing; j++) {
                Field f;
                WD_TRY(alloc_field(c, ring_name(j), lane_s.sp, 1, cap, &f));
                lane_s.Pr.push_back(f);
            }
        if (!mixed) lane_s = lane_d;
        if (hbuf) (void)hipHostFree(hbuf);
        hbuf = nullptr;
        WD_HIP(hipHostMalloc((void **)&hbuf, sizeof(double) * cap, hipHostMallocDefault));
        return WD_OK;
    }

    // Change the number of slots to ncap, keeping the state of slots below
    // min(cap, ncap); slots at or above ncap must be free.  Every new buffer
    // is allocated before any old one is released, so WD_ERR_OOM leaves the
    // solver as it was.
    wd_status resize(int ncap)
    {
        if (ncap == cap) return WD_OK;
        for (int j = ncap; j < cap; j++)
            if (state[j] != SLOT_FREE) return set_error(WD_ERR_STATE, "slot %d is in use", j);
        struct Spec {
            std::string name;
            size_t per_slot;
            int kind;  // 0: rows of per_slot bytes; 1: kScalars arrays of cap doubles; 2: scratch
        };
        std::vector<Spec> sp_list = {{nm("scal"), sizeof(double) * kScalars, 1},
                                     {nm("partial"), sizeof(double) * pstride * 2, 2},
                                     {nm("ids"), sizeof(int) * 3, 2},
                                     {nm("b"), (size_t)b64.rs, 0},
                                     {nm("x"), (size_t)x64.rs, 0},
                                     {nm("r"), (size_t)r64.rs, 0},
                                     {nm("to"), (size_t)to64.rs, 0},
                                     {nm("te"), (size_t)te64.rs, 0},
                                     {nm("ap"), (size_t)Ap64.rs, 0},
                                     {nm("p"), (size_t)p64.rs, 0}};
        if (mixed)
            for (auto f : {std::make_pair("ps", &ps), std::make_pair("rs", &rs), std::make_pair("t2s", &t2s),
                           std::make_pair("tos", &tos), std::make_pair("xs", &xs)})
                sp_list.push_back({nm(f.first), (size_t)f.second->rs, 0});
        // ring slots hold no state across steps (the solution is flushed at
        // every step's end, and the direction is back in slot 0), nor does
        // the alpha history
        const Lane &RL = mixed ? lane_s : lane_d;
        for (int j = 1; j < (int)RL.Pr.size(); j++) sp_list.push_back({ring_name(j), (size_t)RL.Pr[j].rs, 2});
        sp_list.push_back({nm("ahist"), sizeof(double) * kRing, 2});
        const hipStream_t s = c->stream;
        WD_HIP(hipStreamSynchronize(s));
        std::vector<void *> fresh(sp_list.size(), nullptr);
        for (size_t i = 0; i < sp_list.size(); i++) {
            if (hipMalloc(&fresh[i], sp_list[i].per_slot * ncap) != hipSuccess) {
                (void)hipGetLastError();
                for (size_t q = 0; q < i; q++) (void)hipFree(fresh[q]);
                return set_error(WD_ERR_OOM, "session resize to %d slots: device allocation failed", ncap);
            }
        }
        const int keep = std::min(cap, ncap);
        for (size_t i = 0; i < sp_list.size(); i++) {
            auto it = c->ws.find(sp_list[i].name);
            char *old = (char *)it->second.first;
            if (sp_list[i].kind == 0 && keep > 0) {
                WD_HIP(hipMemcpyAsync(fresh[i], old, sp_list[i].per_slot * keep, hipMemcpyDeviceToDevice, s));
            } else if (sp_list[i].kind == 1 && keep > 0) {
                for (int a = 0; a < kScalars; a++)
                    WD_HIP(hipMemcpyAsync((double *)fresh[i] + (size_t)a * ncap, (double *)old + (size_t)a * cap,
                                          sizeof(double) * keep, hipMemcpyDeviceToDevice, s));
            }
        }
        WD_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < sp_list.size(); i++) {
            auto it = c->ws.find(sp_list[i].name);
            (void)hipFree(it->second.first);
            it->second = {fresh[i], sp_list[i].per_slot * ncap};
        }
        WD_TRY(bind(ncap));
        state.resize(cap, SLOT_FREE);
        iters.resize(cap, 0);
        iters64.resize(cap, 0);
        rus.resize(cap, 0);
        status.resize(cap, WD_OK);
        last_ru.resize(cap, 0);
        stall.resize(cap, 0);
        bbh.resize(cap, 0.0);
        maxrr.resize(cap, 0.0);
        best.resize(cap, 0.0);
        tres.resize(cap, 0.0);
        kap.resize(cap, 0.0);
        WD_TRY(upload_list(active, act));
        WD_TRY(upload_list(active64, act64));
        return WD_OK;
    }

    void release()
    {
        if (hbuf) (void)hipHostFree(hbuf);
        hbuf = nullptr;
        for (auto it = c->ws.begin(); it != c->ws.end();) {
            if (it->first.compare(0, pre.size(), pre) == 0) {
                (void)hipFree(it->second.first);
                it = c->ws.erase(it);
            } else {
                ++it;
            }
        }
    }

    wd_status upload_list(const std::vector<int> &v, int *dev)
    {
        if (v.empty()) return WD_OK;
        void *h;
        WD_HIP(hipStreamSynchronize(c->stream));
        WD_TRY(pinned_get(c, 0, sizeof(int) * v.size(), &h));
        std::memcpy(h, v.data(), sizeof(int) * v.size());
        WD_HIP(hipMemcpyAsync(dev, h, sizeof(int) * v.size(), hipMemcpyHostToDevice, c->stream));
        WD_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }

    wd_status upload_coefs()
    {
        std::vector<double> h(2 * cap);
        for (int j = 0; j < cap; j++) {
            h[j] = -kap[j];
            h[cap + j] = -kap[j] * kap[j];
        }
        void *hp;
        WD_HIP(hipStreamSynchronize(c->stream));
        WD_TRY(pinned_get(c, 0, sizeof(double) * 2 * cap, &hp));
        std::memcpy(hp, h.data(), sizeof(double) * 2 * cap);
        WD_HIP(hipMemcpyAsync(coef1, hp, sizeof(double) * 2 * cap, hipMemcpyHostToDevice, c->stream));
        WD_HIP(hipStreamSynchronize(c->stream));
        return WD_OK;
    }

    // out = A in (FP64 or sloppy) for the listed RHS, temporaries to64, te64
    wd_status apply_A(int spp, int lkk, const Field &in, const Field &out, const int *ids, int n, bool norm)
    {
        Sweep sw;
        sw.sp = spp;
        sw.lk = lkk;
        sw.active = ids;
        sw.nact = n;
        if (p.eo) {
            sw.coef = coef2;
            sw.P = 1; sw.dag = 0; sw.epi = EPI_PLAIN; sw.in = in; sw.out = to64;
            WD_TRY(run_sweep(c, sw, nullptr));
            sw.P = 0; sw.epi = EPI_XPAY; sw.in = to64; sw.x = in; sw.out = te64;
            sw.partial = norm ? partial : nullptr; sw.pstride = pstride; sw.pw_off = 0;
            WD_TRY(run_sweep(c, sw, nullptr));
            sw.partial = nullptr;
            sw.P = 1; sw.dag = 1; sw.epi = EPI_PLAIN; sw.in = te64; sw.out = to64;
            WD_TRY(run_sweep(c, sw, nullptr));
            sw.P = 0; sw.epi = EPI_XPAY; sw.in = to64; sw.x = te64; sw.out = out;
            WD_TRY(run_sweep(c, sw, nullptr));
        } else {
            const Field &T = te64;
            sw.coef = coef1;
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
                    sw.partial = (norm && pass == 0) ? partial : nullptr;
                    sw.pstride = pstride;
                    sw.pw_off = P * nw1;
                    WD_TRY(run_sweep(c, sw, nullptr));
                }
            }
        }
        return WD_OK;
    }

    // Ring slots of a lane (1 for the full-lattice iteration).
    static int ring_of(const Lane &L) { return (int)L.Pr.size(); }

    // One CG iteration of the listed RHS of a lane (see the file header):
    // iteration j of the lane's ring cycle; flush: the p update advances the
    // solution by the directions of iterations 0..j and puts the new
    // direction back in slot 0.
    wd_status iterate(const Lane &L, const int *ids, int n, int j, bool flush)
    {
        const hipStream_t s = c->stream;
        if (p.eo) {
            const Field &Pj = L.Pr[j];
            Sweep sw;
            sw.sp = L.sp; sw.lk = L.lk; sw.active = ids; sw.nact = n;
            sw.coef = coef2;
            sw.P = 1; sw.dag = 0; sw.epi = EPI_PLAIN; sw.in = Pj; sw.out = L.TO;
            WD_TRY(run_sweep(c, sw, nullptr));
            sw.P = 0; sw.epi = EPI_XPAY; sw.in = L.TO; sw.x = Pj; sw.out = L.T2;
            sw.partial = partial; sw.pstride = pstride; sw.pw_off = 0;
            WD_TRY(run_sweep(c, sw, nullptr));
            // sweep 3 does not use alpha: it finalizes alpha = rr / p.Ap of
            // sweep 2's partials in extra work-groups while it runs, for
            // sweep 4 (one dispatch fewer than a separate finalize)
            sw.partial = nullptr;
            sw.P = 1; sw.dag = 1; sw.epi = EPI_PLAIN; sw.in = L.T2; sw.out = L.TO;
            if (fold) {
                sw.fin_partial = partial; sw.fin_nw = nwD; sw.fin_pstride = pstride;
                sw.fin_rr = rr; sw.fin_alpha = alpha; sw.fin_out = ahist + (size_t)j * cap;
            } else {
                HIPCHK(blas_finalize(partial, pstride, nwD, ids, n, FIN_ALPHA, rr, alpha, beta,
                                     ahist + (size_t)j * cap, s));
            }
            WD_TRY(run_sweep(c, sw, nullptr));
            sw.fin_partial = nullptr;
            sw.P = 0; sw.epi = EPI_CGUPD; sw.in = L.TO; sw.x = L.T2; sw.r = L.R;
            sw.alpha = alpha; sw.partial = partial;
            WD_TRY(run_sweep(c, sw, nullptr));
            HIPCHK(blas_finalize(partial, pstride, nw1, ids, n, FIN_BETA, rr, alpha, beta, nullptr, s));
            if (flush)
                HIPCHK(blas_p_update_ring(L.Pr.data(), j + 1, L.Pr[0], L.R, beta, true, L.X, ahist, cap, Vh, ids,
                                          n, s));
            else
                HIPCHK(blas_p_update_ring(&L.Pr[j], 1, L.Pr[j + 1], L.R, beta, false, L.X, ahist, cap, Vh, ids,
                                          n, s));
        } else {
            WD_TRY(apply_A(L.sp, L.lk, L.P, Ap64, ids, n, true));
            HIPCHK(blas_finalize(partial, pstride, nwD, ids, n, FIN_ALPHA, rr, alpha, beta, nullptr, s));
            HIPCHK(blas_cg_update(L.X, L.P, L.R, Ap64, alpha, Vh, ids, n, partial, pstride, s));
            HIPCHK(blas_finalize(partial, pstride, nwF, ids, n, FIN_BETA, rr, alpha, beta, nullptr, s));
            HIPCHK(blas_p_update(L.P, L.R, beta, Vh, ids, n, s));
        }
        return WD_OK;
    }

    // The k iterations of a step on both lanes: iteration kk is slot kk mod
    // ring of each lane's cycle; a lane flushes at the end of its ring and at
    // the step's end.
    wd_status iterate_step(int k, int nact, int nact64)
    {
        for (int kk = 0; kk < k; kk++) {
            if (nact) {
                const int R = ring_of(lane_s), j = kk % R;
                WD_TRY(iterate(lane_s, act, nact, j, j == R - 1 || kk == k - 1));
            }
            if (nact64) {
                const int R = ring_of(lane_d), j = kk % R;
                WD_TRY(iterate(lane_d, act64, nact64, j, j == R - 1 || kk == k - 1));
            }
        }
        return WD_OK;
    }

    // Pack n right-hand sides (phi: [n][sites][4][3], device) into free slots
    // and initialise their CG state.  slots_out (host) receives the slots.
    wd_status add(const double *phi, int n, const double *kappa, int *slots_out, const double *x0 = nullptr)
    {
        std::vector<int> slots;
        for (int j = 0; j < cap && (int)slots.size() < n; j++)
            if (state[j] == SLOT_FREE) slots.push_back(j);
        if ((int)slots.size() < n) return set_error(WD_ERR_OOM, "%d free slots, %d requested", (int)slots.size(), n);
        const hipStream_t s = c->stream;
        const long long site_doubles = (long long)24 * Vh * nsub;
        for (int q = 0; q < n; q++) {
            Field v = b64;
            v.base = b64.base + slots[q] * b64.rs;
            HIPCHK(pack_spinor(phi + q * site_doubles, v, 1, p.eo ? 0 : 1, c->g, s));
            kap[slots[q]] = kappa[q];
        }
        WD_TRY(upload_coefs());
        WD_TRY(upload_list(slots, lst));
        HIPCHK(blas_norm(b64, Vh, lst, n, partial, pstride, s));
        HIPCHK(blas_finalize(partial, pstride, nwF, lst, n, FIN_STORE, rr, alpha, beta, bb, s));
        if (x0) {
            // start from x0: x = x0, r = b - A x0 in FP64, rr = |r|^2
            for (int q = 0; q < n; q++) {
                Field v = x64;
                v.base = x64.base + slots[q] * x64.rs;
                HIPCHK(pack_spinor(x0 + q * site_doubles, v, 1, p.eo ? 0 : 1, c->g, s));
            }
            WD_TRY(apply_A(SP_F64, c->lk64, x64, Ap64, lst, n, false));
            HIPCHK(blas_resid(r64, b64, Ap64, Vh, lst, n, partial, pstride, s));
        } else {
            HIPCHK(blas_zero(x64, Vh, lst, n, s));
            HIPCHK(blas_copy(r64, b64, Vh, lst, n, s));
        }
        HIPCHK(blas_finalize(partial, pstride, nwF, lst, n, FIN_RR, rr, alpha, beta, nullptr, s));
        if (mixed) {
            HIPCHK(blas_copy(rs, r64, Vh, lst, n, s));
            HIPCHK(blas_zero(xs, Vh, lst, n, s));
        }
        HIPCHK(blas_copy(lane_s.P, lane_s.R, Vh, lst, n, s));
        std::vector<double> rr0(cap, 0.0);
        HIPCHK(hipMemcpyAsync(hbuf, rr, sizeof(double) * cap, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int q = 0; q < n; q++) rr0[slots[q]] = hbuf[slots[q]];
        HIPCHK(hipMemcpyAsync(hbuf, bb, sizeof(double) * cap, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double tol2 = p.tol * p.tol;
        for (int q = 0; q < n; q++) {
            const int j = slots[q];
            bbh[j] = hbuf[j];
            iters[j] = iters64[j] = 0;
            rus[j] = 0;
            last_ru[j] = 0;
            stall[j] = 0;
            tres[j] = 0.0;
            maxrr[j] = best[j] = rr0[j];
            if (!std::isfinite(bbh[j]) || !std::isfinite(rr0[j])) {
                state[j] = SLOT_DONE;
                status[j] = WD_ERR_NAN;
                tres[j] = NAN;
            } else if (bbh[j] == 0.0 && rr0[j] == 0.0) {
                state[j] = SLOT_DONE;
                status[j] = WD_OK;
            } else if (rr0[j] <= tol2 * bbh[j]) {  // the initial guess already meets tol
                state[j] = SLOT_DONE;
                status[j] = WD_OK;
                tres[j] = std::sqrt(rr0[j] / bbh[j]);
            } else {
                state[j] = SLOT_RUNNING;
                status[j] = WD_ERR_NOCONV;
                active.push_back(j);
            }
            if (slots_out) slots_out[q] = j;
        }
        std::sort(active.begin(), active.end());
        WD_TRY(upload_list(active, act));
        return WD_OK;
    }

    // Reliable update of the listed RHS of a lane: (sloppy lane) x64 += X,
    // X = 0; r64 = b - A x64 in FP64, rr = |r64|^2, R = r64.  The search
    // direction P = R_old + beta_old p_prev was built from the replaced
    // recursive residual R_old, beta_old = |R_old|^2 / |r_prev|^2; it is
    // rebuilt with the true residual: q = P - R_old is made orthogonal to r64
    // and P = r64 + (|r64|^2 / |R_old|^2) q, which is beta = |r64|^2 /
    // |r_prev|^2 (as in reliable-update CG, Clark et al. 2010).  rrh[j]
    // receives the new |r|^2.
    wd_status reliable(const Lane &L, const std::vector<int> &ids, std::vector<double> &rrh)
    {
        if (ids.empty()) return WD_OK;
        const hipStream_t s = c->stream;
        WD_TRY(upload_list(ids, lst));
        const int n = (int)ids.size();
        HIPCHK(hipMemcpyAsync(rr_s, rr, sizeof(double) * cap, hipMemcpyDeviceToDevice, s));
        HIPCHK(blas_axpy_const(L.P, L.R, -1.0, Vh, lst, n, s));
        if (L.sloppy) HIPCHK(blas_add_zero(x64, L.X, Vh, lst, n, s));
        WD_TRY(apply_A(SP_F64, c->lk64, x64, Ap64, lst, n, false));
        HIPCHK(blas_resid(r64, b64, Ap64, Vh, lst, n, partial, pstride, s));
        HIPCHK(blas_finalize(partial, pstride, nwF, lst, n, FIN_RR, rr, alpha, beta, nullptr, s));
        if (L.sloppy) HIPCHK(blas_copy(L.R, r64, Vh, lst, n, s));
        HIPCHK(blas_cdot(L.R, L.P, Vh, lst, n, partial, partial2, pstride, s));
        HIPCHK(blas_finalize(partial, pstride, nwF, lst, n, FIN_STORE, rr, alpha, beta, dre, s));
        HIPCHK(blas_finalize(partial2, pstride, nwF, lst, n, FIN_STORE, rr, alpha, beta, dim, s));
        HIPCHK(blas_orth(L.P, L.R, dre, dim, rr, Vh, lst, n, s));
        HIPCHK(blas_xpay_ratio(L.P, L.R, rr, rr_s, Vh, lst, n, s));
        HIPCHK(hipMemcpyAsync(hbuf, rr, sizeof(double) * cap, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int j : ids) rrh[j] = hbuf[j];
        return WD_OK;
    }

    // Everything the kernel arguments of a step depend on: field and scalar
    // addresses and strides, RHS counts (grid sizes), formats, launch shapes.
    std::string graph_key(int k, int nact, int nact64) const
    {
        std::string key = pre;
        auto add = [&key](unsigned long long v) {
            key += '|';
            key += std::to_string(v);
        };
        auto addf = [&add](const Field &f) {
            add((unsigned long long)(uintptr_t)f.base);
            add((unsigned long long)f.rs);
            add((unsigned long long)f.ss);
            add((unsigned long long)f.sp);
            add((unsigned long long)f.nsub);
            add((unsigned long long)f.cs);
        };
        for (unsigned long long v : {(unsigned long long)k, (unsigned long long)nact, (unsigned long long)nact64,
                                     (unsigned long long)c->use_tuned, (unsigned long long)c->tune_gen,
                                     (unsigned long long)sp, (unsigned long long)lk, (unsigned long long)xp,
                                     (unsigned long long)c->lk64, (unsigned long long)p.eo,
                                     (unsigned long long)pstride, (unsigned long long)fold})
            add(v);
        for (const void *q : {(const void *)c->links64, (const void *)c->links32, (const void *)c->links16,
                              (const void *)c->links32r, (const void *)c->links8, (const void *)coef1,
                              (const void *)coef2,
                              (const void *)rr, (const void *)alpha, (const void *)beta, (const void *)partial,
                              (const void *)act, (const void *)act64, (const void *)ahist})
            add((unsigned long long)(uintptr_t)q);
        add((unsigned long long)cap);
        for (const Lane *L : {&lane_s, &lane_d}) {
            addf(L->P);
            addf(L->R);
            addf(L->T2);
            addf(L->TO);
            addf(L->X);
            add((unsigned long long)L->Pr.size());
            for (const Field &f : L->Pr) addf(f);
        }
        addf(Ap64);
        return key;
    }

    // The k iterations of a step as one HIP graph: captured on the context's
    // private stream the first time this key is seen, then replayed on the
    // context's stream.  The graph holds kernel launches only (no memsets).
    wd_status run_graph(int k, int nact, int nact64)
    {
        const std::string key = graph_key(k, nact, nact64);
        hipGraphExec_t ex = nullptr;
        for (auto &g : c->graphs)
            if (g.first == key) ex = g.second;
        if (!ex) {
            if (!c->capture_stream)
                WD_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            const hipStream_t saved = c->stream;
            WD_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
            c->stream = c->capture_stream;
            const wd_status st = iterate_step(k, nact, nact64);
            c->stream = saved;
            hipGraph_t gph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->capture_stream, &gph);
            if (st != WD_OK) {
                if (gph) (void)hipGraphDestroy(gph);
                return st;
            }
            if (e != hipSuccess || !gph) return set_error(WD_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
            const hipError_t e2 = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gph);
            if (e2 != hipSuccess) return set_error(WD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e2));
            if (c->graphs.size() >= kMaxGraphs) {
                (void)hipGraphExecDestroy(c->graphs.front().second);
                c->graphs.erase(c->graphs.begin());
            }
            c->graphs.push_back({key, ex});
        }
        WD_HIP(hipGraphLaunch(ex, c->stream));
        return WD_OK;
    }

    // k iterations of every running RHS, then the residual checks.
    wd_status step(int k)
    {
        if ((active.empty() && active64.empty()) || k < 1) return WD_OK;
        const hipStream_t s = c->stream;
        const int nact = (int)active.size(), nact64 = (int)active64.size();
        if (p.graphs && !c->timing) {
            WD_TRY(run_graph(k, nact, nact64));
        } else {
            WD_TRY(iterate_step(k, nact, nact64));
        }
        for (int j : active) iters[j] += k;
        for (int j : active64) {
            iters[j] += k;
            iters64[j] += k;
        }
        HIPCHK(hipMemcpyAsync(hbuf, rr, sizeof(double) * cap, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double tol2 = p.tol * p.tol, d2 = p.delta * p.delta;
        std::vector<double> rrh(cap, 0.0), r2s(cap, 0.0);
        std::vector<int> ru[2], keep[2];
        for (int l = 0; l < 2; l++) {
            const bool sl = l == 0 && mixed;  // a sloppy lane with FP64 updates
            for (int j : (l == 0 ? active : active64)) {
                const double r2 = hbuf[j];
                r2s[j] = r2;
                if (trace) fprintf(stderr, "[wd cg] it %d rhs %d %s |r|/|b| %.3e\n", iters[j], j,
                                   l ? "fp64" : "sloppy", std::sqrt(r2 / bbh[j]));
                if (!std::isfinite(r2)) {
                    status[j] = WD_ERR_NAN;
                    tres[j] = NAN;
                    state[j] = SLOT_DONE;
                    continue;
                }
                const bool at_cap = iters[j] >= p.maxiter;
                if (r2 <= tol2 * bbh[j] || at_cap ||
                    (sl && (r2 < d2 * maxrr[j] || iters[j] - last_ru[j] >= kMaxItersPerUpdate)))
                    ru[l].push_back(j);
                if (r2 > maxrr[j]) maxrr[j] = r2;
                keep[l].push_back(j);
            }
        }
        WD_TRY(reliable(lane_s, ru[0], rrh));
        WD_TRY(reliable(lane_d, ru[1], rrh));
        std::vector<int> restart[2], escalate;
        for (int l = 0; l < 2; l++) {
            std::vector<int> keep2;
            for (int j : keep[l]) {
                bool done = false, moved = false;
                if (std::find(ru[l].begin(), ru[l].end(), j) != ru[l].end()) {
                    rus[j]++;
                    last_ru[j] = iters[j];
                    if (trace)
                        fprintf(stderr, "[wd cg] it %d rhs %d reliable update: true |r|/|b| %.3e\n", iters[j], j,
                                std::sqrt(rrh[j] / bbh[j]));
                    if (!std::isfinite(rrh[j])) {
                        status[j] = WD_ERR_NAN;
                        tres[j] = NAN;
                        done = true;
                    } else if (rrh[j] <= tol2 * bbh[j]) {
                        status[j] = WD_OK;
                        tres[j] = std::sqrt(rrh[j] / bbh[j]);
                        done = true;
                    } else if (iters[j] >= p.maxiter) {
                        status[j] = WD_ERR_NOCONV;
                        tres[j] = std::sqrt(rrh[j] / bbh[j]);
                        done = true;
                    } else {
                        maxrr[j] = rrh[j];
                        if (rrh[j] < best[j]) {
                            best[j] = rrh[j];
                            stall[j] = 0;
                        } else {
                            stall[j]++;
                        }
                        if (l == 0 && mixed && stall[j] >= kStallUpdates) {
                            escalate.push_back(j);
                            moved = true;
                        } else if (rrh[j] > kDriftRestart * r2s[j]) {
                            restart[l].push_back(j);
                        }
                    }
                }
                if (done)
                    state[j] = SLOT_DONE;
                else if (!moved)
                    keep2.push_back(j);
            }
            keep[l].swap(keep2);
        }
        // restarts p = r; escalated slots start FP64 CG from p64 = r64 (the
        // true residual of their current x64)
        if (!restart[0].empty()) {
            WD_TRY(upload_list(restart[0], lst));
            HIPCHK(blas_copy(lane_s.P, lane_s.R, Vh, lst, (int)restart[0].size(), s));
        }
        for (int j : escalate) restart[1].push_back(j);
        if (!restart[1].empty()) {
            WD_TRY(upload_list(restart[1], lst));
            HIPCHK(blas_copy(p64, r64, Vh, lst, (int)restart[1].size(), s));
        }
        if (trace) {
            for (int l = 0; l < 2; l++)
                for (int j : restart[l]) fprintf(stderr, "[wd cg] it %d rhs %d restart p = r\n", iters[j], j);
            for (int j : escalate) fprintf(stderr, "[wd cg] it %d rhs %d continues in FP64\n", iters[j], j);
        }
        for (int j : escalate) keep[1].push_back(j);
        std::sort(keep[1].begin(), keep[1].end());
        if (keep[0] != active) {
            active.swap(keep[0]);
            WD_TRY(upload_list(active, act));
        }
        if (keep[1] != active64) {
            active64.swap(keep[1]);
            WD_TRY(upload_list(active64, act64));
        }
        return WD_OK;
    }

    bool running() const { return !active.empty() || !active64.empty(); }

    wd_status unpack(int slot, double *x)
    {
        Field v = x64;
        v.base = x64.base + slot * x64.rs;
        HIPCHK(unpack_spinor(v, x, 1, p.eo ? 0 : 1, c->g, c->stream));
        return WD_OK;
    }

    void fill_stats(int j, double secs, wd_solver_stats *st) const
    {
        st->iters = iters[j];
        st->reliable_updates = rus[j];
        st->true_resid = tres[j];
        st->seconds = secs;
        st->status = status[j];
        st->iters_fp64 = mixed ? iters64[j] : iters[j];
    }
};

static wd_status check_params(const wd_solver_params &p)
{
    if (!(p.tol > 0) || p.maxiter < 0 || p.poll < 1 || !(p.delta > 0 && p.delta < 1))
        return set_error(WD_ERR_ARG, "bad solver parameters (tol %g maxiter %d poll %d delta %g)", p.tol,
                         p.maxiter, p.poll, p.delta);
    return WD_OK;
}

}  // namespace wd

using namespace wd;

struct wd_session {
    BatchSolver bs;
    std::chrono::steady_clock::time_point t0;
};

namespace {
struct TunedScope {
    wd_ctx *c;
    bool old;
    ~TunedScope() { c->use_tuned = old; }
};
}  // namespace

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
    WD_TRY(check_params(p));
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(kappa[j])) return set_error(WD_ERR_ARG, "kappa[%d] not finite", j);
    WD_HIP(hipSetDevice(c->device));
    TunedScope tscope{c, c->use_tuned};
    c->use_tuned = p.tuned != 0;

    // the one-shot solver keeps its state in the context's "cg_" workspaces,
    // reused across calls; only its pinned buffer is released here
    BatchSolver bs;
    struct PinnedScope {
        BatchSolver &b;
        ~PinnedScope()
        {
            if (b.hbuf) (void)hipHostFree(b.hbuf);
        }
    } pscope{bs};
    WD_TRY(bs.init(c, nrhs, p, "cg_"));
    WD_TRY(bs.add(phi, nrhs, kappa, nullptr, p.initial_guess ? x : nullptr));
    int it = 0;
    while (bs.running() && it < p.maxiter) {
        const int k = std::min(p.poll, p.maxiter - it);
        WD_TRY(bs.step(k));
        it += k;
    }
    for (int j = 0; j < nrhs; j++)  // only when maxiter = 0
        if (bs.state[j] == SLOT_RUNNING) {
            bs.status[j] = WD_ERR_NOCONV;
            bs.state[j] = SLOT_DONE;
        }
    for (int j = 0; j < nrhs; j++) WD_TRY(bs.unpack(j, x + (size_t)j * 24 * c->Vh * bs.nsub));
    WD_HIP(hipStreamSynchronize(c->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    wd_status ret = WD_OK;
    for (int j = 0; j < nrhs; j++) {
        if (st) bs.fill_stats(j, secs, &st[j]);
        if (bs.status[j] == WD_ERR_NAN) ret = WD_ERR_NAN;
        else if (bs.status[j] != WD_OK && ret == WD_OK) ret = (wd_status)bs.status[j];
    }
    if (ret != WD_OK) set_error(ret, "%s", ret == WD_ERR_NAN ? "non-finite residual" : "not converged");
    return ret;
}

static std::atomic<unsigned> g_session_id{0};

extern "C" wd_status wd_session_create(wd_ctx *c, int max_rhs, const wd_solver_params *pin, wd_session **out)
{
    if (!c || !out) return set_error(WD_ERR_ARG, "NULL argument");
    if (max_rhs < 1 || max_rhs > 1024) return set_error(WD_ERR_ARG, "max_rhs %d out of range", max_rhs);
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    wd_solver_params p;
    wd_solver_defaults(&p);
    if (pin) p = *pin;
    WD_TRY(check_params(p));
    WD_HIP(hipSetDevice(c->device));
    wd_session *s = new wd_session();
    char pre[32];
    snprintf(pre, sizeof(pre), "ses%u_", g_session_id.fetch_add(1));
    wd_status st = s->bs.init(c, max_rhs, p, pre);
    if (st != WD_OK) {
        s->bs.release();
        delete s;
        return st;
    }
    s->t0 = std::chrono::steady_clock::now();
    c->sessions++;
    *out = s;
    return WD_OK;
}

extern "C" wd_status wd_session_destroy(wd_session *s)
{
    if (!s) return WD_OK;
    wd_ctx *c = s->bs.c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    s->bs.release();
    delete s;
    c->sessions--;
    return WD_OK;
}

extern "C" wd_status wd_session_add(wd_session *s, const double *phi, int nrhs, const double *kappa,
                                    int32_t *slots)
{
    if (!s || !phi || !kappa || nrhs < 1) return set_error(WD_ERR_ARG, "bad argument");
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(kappa[j])) return set_error(WD_ERR_ARG, "kappa[%d] not finite", j);
    WD_HIP(hipSetDevice(s->bs.c->device));
    std::vector<int> sl(nrhs);
    WD_TRY(s->bs.add(phi, nrhs, kappa, sl.data()));
    if (slots)
        for (int j = 0; j < nrhs; j++) slots[j] = sl[j];
    return WD_OK;
}

extern "C" wd_status wd_session_step(wd_session *s, int k_iters)
{
    if (!s || k_iters < 1) return set_error(WD_ERR_ARG, "bad argument");
    wd_ctx *c = s->bs.c;
    WD_HIP(hipSetDevice(c->device));
    TunedScope tscope{c, c->use_tuned};
    c->use_tuned = s->bs.p.tuned != 0;
    return s->bs.step(k_iters);
}

extern "C" wd_status wd_session_resize(wd_session *s, int max_rhs)
{
    if (!s) return set_error(WD_ERR_ARG, "NULL session");
    if (max_rhs < 1 || max_rhs > 1024) return set_error(WD_ERR_ARG, "max_rhs %d out of range", max_rhs);
    WD_HIP(hipSetDevice(s->bs.c->device));
    return s->bs.resize(max_rhs);
}

extern "C" int wd_session_capacity(const wd_session *s) { return s ? s->bs.cap : 0; }

extern "C" wd_status wd_session_poll(wd_session *s, int32_t *state, wd_solver_stats *st)
{
    if (!s) return set_error(WD_ERR_ARG, "NULL session");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
    for (int j = 0; j < s->bs.cap; j++) {
        if (state) state[j] = s->bs.state[j];
        if (st) s->bs.fill_stats(j, secs, &st[j]);
    }
    return WD_OK;
}

extern "C" wd_status wd_session_take(wd_session *s, int slot, double *x)
{
    if (!s || !x) return set_error(WD_ERR_ARG, "NULL argument");
    if (slot < 0 || slot >= s->bs.cap) return set_error(WD_ERR_ARG, "slot %d out of range", slot);
    if (s->bs.state[slot] != SLOT_DONE) return set_error(WD_ERR_STATE, "slot %d is not done", slot);
    WD_HIP(hipSetDevice(s->bs.c->device));
    WD_TRY(s->bs.unpack(slot, x));
    WD_HIP(hipStreamSynchronize(s->bs.c->stream));
    s->bs.state[slot] = SLOT_FREE;
    return WD_OK;
}

extern "C" size_t wd_session_bytes(const int32_t dims[4], int max_rhs, const wd_solver_params *p)
{
    // the solver state of max_rhs slots, without the gauge field
    const size_t all = wd_bytes_required(dims, max_rhs, p), gauge = wd_bytes_required(dims, 0, p);
    return all > gauge ? all - gauge : 0;
}
