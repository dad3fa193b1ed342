/*
 * wd.h -- C-ABI of the MI355X (gfx950) Wilson-Dirac / CG / HMC library.
 *
 * The operations follow arXiv:1207.2223 ("Hybrid Monte Carlo with Wilson Dirac
 * operator on the Fermi GPU"): the fermion matrix M = D + m applied to a
 * pseudofermion field and its adjoint (Sec. 3, kernel 1), the conjugate-gradient
 * inversion of M^dag M that the pseudofermion action of eq. (4) requires
 * (eq. 3 and Sec. 2), the molecular-dynamics force (Sec. 3, kernels 2 and 3)
 * and the HMC trajectory of Sec. 3 (refresh, leapfrog, accept/reject).
 *
 * Conventions shared by every call
 * --------------------------------
 *  lattice  dims = {Lx, Ly, Lz, Lt}, every extent even and >= 2; periodic
 *           boundaries in all four directions for links and fermions.
 *           lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) & 1;
 *           checkerboard index cb = lex >> 1; V = Lx*Ly*Lz*Lt, Vh = V/2.
 *  operator M = 1 - kappa*H (the kappa-normalised M = D + m, eq. 4) with
 *           (H psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
 *                              + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu),
 *           gamma matrices in the chiral (DeGrand-Rossi) basis, gamma_1..4
 *           along x, y, z, t.  M^dag = 1 - kappa*H^dag swaps (1-g) and (1+g).
 *           Even-odd: D_eo / D_oe are the parity blocks of H and
 *           Mhat = 1 - kappa^2 D_eo D_oe acts on even sites.
 *  layouts  canonical complex128 with interleaved (re, im) doubles:
 *             full spinor   [V][4 spin][3 colour]      lex order
 *             parity spinor [Vh][4][3]                 cb order of that parity
 *             links         [V][4 mu][3][3]            U_mu(x), row-major
 *             momenta/force [V][4][3][3]               Hermitian traceless
 *           Batches of right-hand sides are [nrhs][...] back to back.
 *  memory   Unless stated otherwise, every pointer argument is a DEVICE
 *           pointer on the context's device (e.g. a torch tensor's
 *           data_ptr()), owned by the caller and never retained after the
 *           call returns.  The library owns its packed copy of the gauge
 *           field and all workspaces.
 *  streams  Work is issued on the hipStream_t given to wd_create.  Calls
 *           that return statistics synchronise that stream before returning.
 *  errors   Every call returns a wd_status; on failure wd_last_error()
 *           returns a message for the calling thread.  WD_ERR_ARG,
 *           WD_ERR_DIMS and WD_ERR_OOM are raised before any output is
 *           written.
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WD_OK = 0,
    WD_ERR_ARG = -1,    /* invalid argument (null pointer, bad enum, bad size) */
    WD_ERR_DIMS = -2,   /* lattice extent odd, < 2, or too large               */
    WD_ERR_OOM = -3,    /* device allocation failed or budget exceeded         */
    WD_ERR_HIP = -4,    /* a HIP runtime call failed                           */
    WD_ERR_NOCONV = -5, /* solver hit maxiter; best iterate is returned        */
    WD_ERR_NAN = -6,    /* non-finite residual or breakdown (p.Ap <= 0)        */
    WD_ERR_STATE = -7   /* call out of order (e.g. no gauge field loaded)      */
} wd_status;

/* Sloppy spinor formats: FP64, FP32, FP16 with a per-site FP32 norm, and
 * int16 fixed point with a per-site FP32 norm (q = rint(v * 32767 / n), n =
 * max |v| over the site's 24 reals; 52 bytes per site like FP16; FP32
 * arithmetic; 12-real FP32 or FP16 links). */
typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2, WD_I16 = 3 } wd_prec;
/* Or-ed into a WD_F32 / WD_F16 / WD_I16 precision code: the sloppy operator
 * reads FP16 12-real links (WD_LINKS_F16) or FP32 links with all 18 reals
 * (WD_LINKS_R18, no reconstruction; not with WD_I16) instead of FP32 12-real
 * links. */
#define WD_LINKS_F16 0x10
#define WD_LINKS_R18 0x20
/* Or-ed into WD_F32 / WD_F16: FP32 links stored as 8 reals (32 bytes instead
 * of 48; the paper's closing remarks on reconstructing links on the fly): of
 * a column- and row-permuted copy of the link, chosen per link so that the
 * reconstruction is well conditioned, a2, a3, b1 and the phases of a1 and
 * c1; the rest is rebuilt in registers from unitarity and det U = 1.  1 or 2
 * RHS per lane (for sweeps with few RHS, where the link bytes weigh most). */
#define WD_LINKS_R8 0x40
typedef enum { WD_FULL = 0, WD_EVEN = 1, WD_ODD = 2 } wd_parity;

/* wd_gauge_load flags: storage of the FP64 operator's links. */
#define WD_RECON_18 0u /* all 18 reals of each link                        */
#define WD_RECON_12 1u /* rows 1-2 only; row 3 = conj(row1 x row2) on load */

typedef struct wd_ctx wd_ctx;

/* Solver parameters (CG on M^dag M, eq. 3-4). */
typedef struct {
    double tol;       /* target true relative residual |b - A x|_2 / |b|_2 (FP64)  */
    int maxiter;      /* iteration cap; WD_ERR_NOCONV past it                       */
    int prec_sloppy;  /* wd_prec of the iterated operator and vectors               */
    int eo;           /* 1: A = Mhat^dag Mhat on even sites; 0: A = M^dag M (full)  */
    double delta;     /* reliable update when |r| < delta * max|r| since the last  */
    int poll;         /* iterations between host checks of the residual norms       */
    int tuned;        /* 1: use autotuned launch shapes (wd_tune), 0: defaults      */
    int graphs;       /* 1: run the poll iterations of a step as one captured HIP   */
                      /* graph, replayed while the active set is unchanged; 0:    */
                      /* launch each kernel (same results bit for bit)            */
    int initial_guess; /* wd_cg_solve: 1: x holds the starting vectors on entry  */
                      /* (r0 = b - A x in FP64); 0: x0 = 0 (x is output only)     */
} wd_solver_params;

/* Per right-hand-side solver statistics. */
typedef struct {
    int iters;            /* CG iterations applied to this RHS                     */
    int reliable_updates; /* FP64 true-residual recomputations                     */
    double true_resid;    /* final |b - A x| / |b| in FP64                          */
    double seconds;       /* wall time of the whole batched call                   */
    int status;           /* wd_status of this RHS                                 */
    int iters_fp64;       /* of iters, those run in FP64: all of them for an FP64  */
                          /* solve; in a mixed solve, those after the RHS left the */
                          /* sloppy precision because its true residual stalled    */
} wd_solver_stats;

/* Fill p with the defaults: tol 1e-10, maxiter 20000, FP64, eo 1, delta 0.1,
 * poll 8, tuned 0, graphs 1, initial_guess 0.  p: host pointer. */
void wd_solver_defaults(wd_solver_params *p);

/* Create a context for one lattice on HIP device `device`, issuing work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  *c receives the
 * handle.  WD_ERR_DIMS for an odd or too small extent, or V >= 2^31. */
wd_status wd_create(wd_ctx **c, const int32_t dims[4], int device, void *hip_stream);

/* Free the context and everything it owns.  NULL is accepted.  Solver
 * sessions created on it must be destroyed first: WD_ERR_STATE (nothing
 * freed) while any is open. */
wd_status wd_destroy(wd_ctx *c);

/* Bind a different stream for subsequent work (NULL = null stream). */
wd_status wd_set_stream(wd_ctx *c, void *hip_stream);

/* Load the gauge field U (canonical [V][4][3][3] complex128, device) and pack
 * it into the internal layouts: FP64 with 18 or 12 reals (flags), and FP32
 * 12-real, FP32 18-real and FP16 12-real copies for the sloppy operators.  Links are assumed to be
 * in SU(3) (12-real reconstruction is exact only there). */
wd_status wd_gauge_load(wd_ctx *c, const double *U, uint32_t flags);

/* Hopping term (Sec. 3, kernel 1, without the mass term):
 *   out_parity = WD_EVEN / WD_ODD: out[Vh][4][3] = D_{P,1-P} in, with `in`
 *     the [Vh][4][3] field on the other parity;
 *   out_parity = WD_FULL: out[V][4][3] = H in on the full lattice.
 * dagger = 1 applies H^dag.  prec (a wd_prec, optionally | WD_LINKS_F16 or
 * | WD_LINKS_R18)
 * selects the arithmetic and storage used inside: FP64 with the gauge_load
 * link format, or FP32 / FP16-with-norm spinors with FP32 (or FP16) 12-real
 * links and FP32 arithmetic.  The canonical in/out stay FP64. */
wd_status wd_dslash(wd_ctx *c, double *out, const double *in, int out_parity, int dagger,
                    int prec);

/* The parity blocks of the hopping term (as wd_dslash with WD_EVEN / WD_ODD)
 * on nrhs right-hand sides at once (in, out: [nrhs][Vh][4][3], 1..64) with an
 * explicit launch shape of the stencil kernel: shape (HOST int32[5]) =
 * {threads per work-group (64, 128, 192 or 256), RHS per lane, lanes per
 * site, tile order (0..7, as the autotuner's; 8, 9, 10: the LDS-staged
 * kernel walking 4, 8 or 16 t-planes of a z-plane column per work-group, with
 * 256 threads, 1 lane per site, 1 or 2 RHS per lane, no cap, FP16 or FP32
 * spinors, where a plane of one parity holds a multiple of 64 sites up to
 * 512, Lz is a multiple of 8 and Lt of the chunk; 11, 12, 13: the t-walking
 * kernel, each work-group a tile of `threads` sites (64, 128 or 256 dividing
 * the sites of a plane of one parity) walking 4, 8 or 16 t-planes with the t
 * neighbours held in registers, 1 lane per site, 1 to 3 RHS per lane, FP16
 * spinors with FP32 or FP16 12-real links, Lz a multiple of 8 and Lt of the
 * chunk), work-groups per CU cap (0 or 2..8)}, or NULL for the default
 * shape.  Every supported shape gives the
 * same bits; WD_ERR_ARG for a shape this lattice or precision does not
 * support (e.g. a slab tile order when the slab extent is not a multiple of
 * 8).  For checking launch shapes against a reference operator. */
wd_status wd_dslash_shaped(wd_ctx *c, double *out, const double *in, int nrhs, int out_parity, int dagger,
                           int prec, const int32_t shape[5]);

/* Normal operator: eo = 0: out = M^dag M in (full [V][4][3]);
 * eo = 1: out = Mhat^dag Mhat in (even [Vh][4][3]).  FP64 arithmetic. */
wd_status wd_mdagm(wd_ctx *c, double *out, const double *in, double kappa, int eo);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * normal operator as wd_mdagm -- same arguments, same kernels, the same bits
 * -- with its packed operand, temporaries and device scalars in a fixed
 * device array of 64 MiB per GPU (held from the first wd_create on that GPU
 * until the process ends) instead of context workspaces.  The call allocates
 * nothing and copies nothing between host and device.  Lattices whose
 * operator needs more than the 64 MiB (about Vh <= 87000 for eo = 1, Vh <=
 * 58000 for eo = 0; e.g. 16^3 x 32 even-odd fits, its full lattice does not)
 * are refused with WD_ERR_ARG before any work is issued.  Every call on one
 * GPU uses that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller. */
wd_status wd_mdagm_noalloc(wd_ctx *c, double *out, const double *in, double kappa, int eo);

/* Solve A x_j = phi_j for nrhs right-hand sides at once (eq. 3: the inverse
 * of M^dag M applied to the pseudofermion).  A is M^dag M (p->eo = 0, fields
 * [nrhs][V][4][3]) or Mhat^dag Mhat (p->eo = 1, fields [nrhs][Vh][4][3],
 * even sites).  kappa: HOST array [nrhs], one hopping parameter per RHS.
 * st: HOST array [nrhs] or NULL.  x0 = 0.  Converged means the FP64 true
 * residual meets p->tol.  With a sloppy precision the iteration runs in
 * FP32 or FP16 (per-site norm) with FP64 dot products and FP64 reliable
 * updates.  Returns WD_ERR_NOCONV / WD_ERR_NAN if any RHS failed (the other
 * RHS are still solved); x holds the best iterate of every RHS. */
wd_status wd_cg_solve(wd_ctx *c, double *x, const double *phi, int nrhs, const double *kappa,
                      const wd_solver_params *p, wd_solver_stats *st);

/* ---------------------------------------------------------------------- */
/* Solver sessions: persistent batched CG state for continuous batching.     */
/* A session owns the device state of max_rhs slots on one context (one    */
/* lattice and gauge field).  Right-hand sides join between steps; every    */
/* running slot advances k iterations per step; reliable updates and        */
/* convergence are decided from each slot's own history at multiples of k   */
/* of its own iteration count, so a slot's result is bitwise the same alone */
/* or batched with others (for equal k and parameters).  Calls on one       */
/* session (and context) must not overlap; different contexts may run on    */
/* different streams concurrently.                                          */
/* ---------------------------------------------------------------------- */

typedef struct wd_session wd_session;

/* Create a session of max_rhs slots (1..1024) solving with parameters p
 * (NULL = defaults; p->maxiter bounds each slot, p->poll is unused).
 * Allocates the state of max_rhs slots (WD_ERR_OOM if it does not fit);
 * wd_session_resize changes the number later. */
wd_status wd_session_create(wd_ctx *c, int max_rhs, const wd_solver_params *p, wd_session **s);

/* Free the session and its device state (before its context).  NULL is
 * accepted. */
wd_status wd_session_destroy(wd_session *s);

/* Add nrhs right-hand sides phi ([nrhs][sites][4][3] device, sites = Vh for
 * eo, V otherwise) with hopping parameters kappa (HOST [nrhs]); slots (HOST
 * [nrhs], may be NULL) receives the slots used.  WD_ERR_OOM if fewer than
 * nrhs slots are free (nothing is added then).  phi may be freed after the
 * call returns. */
wd_status wd_session_add(wd_session *s, const double *phi, int nrhs, const double *kappa, int32_t *slots);

/* Run k_iters iterations of every running slot, then the residual checks
 * (synchronises the context's stream). */
wd_status wd_session_step(wd_session *s, int k_iters);

/* Change the number of slots to max_rhs (1..1024).  Slots below the smaller
 * of the old and new counts keep their state (running solves continue
 * unchanged, bitwise); shrinking needs every slot >= max_rhs to be free
 * (WD_ERR_STATE otherwise).  The device state is reallocated at the new
 * size, so memory is returned on shrinking.  WD_ERR_OOM leaves the session
 * unchanged.  Synchronises the context's stream. */
wd_status wd_session_resize(wd_session *s, int max_rhs);

/* Current number of slots (0 for NULL). */
int wd_session_capacity(const wd_session *s);

/* Slot states (HOST [wd_session_capacity(s)], 0 free, 1 running, 2 done;
 * may be NULL) and stats (HOST [wd_session_capacity(s)], may be NULL;
 * seconds = time since creation). */
wd_status wd_session_poll(wd_session *s, int32_t *state, wd_solver_stats *st);

/* Copy the solution of a done slot to x ([sites][4][3] device) and free the
 * slot.  WD_ERR_STATE if the slot is not done. */
wd_status wd_session_take(wd_session *s, int slot, double *x);

/* Device bytes of a session of max_rhs slots (without the gauge field). */
size_t wd_session_bytes(const int32_t dims[4], int max_rhs, const wd_solver_params *p);

/* ---------------------------------------------------------------------- */
/* Molecular dynamics and HMC (Sec. 2, eq. 5; Sec. 3 kernels 2-4 and the     */
/* three steps of a trajectory).  Even-odd action                            */
/*   S = beta sum_{x,mu<nu} (1 - Re tr U_munu / 3)                           */
/*     + phi_e^dag (Mhat^dag Mhat)^-1 phi_e,   H = S + 1/2 sum tr p^2.       */
/* ---------------------------------------------------------------------- */

typedef struct {
    double beta;                   /* gauge coupling of the plaquette action          */
    double kappa;                  /* hopping parameter                               */
    double tau;                    /* trajectory length                               */
    int nsteps;                    /* leapfrog steps (P-Q-P), dtau = tau / nsteps      */
    uint32_t traj;                 /* trajectory index: Philox counter word           */
    uint64_t seed;                 /* Philox key                                      */
    wd_solver_params force_solver; /* solves inside the force (eo must be 1)          */
    wd_solver_params h_solver;     /* the final-Hamiltonian solve (eo must be 1)      */
    int metropolis;                /* 1: accept iff u < exp(-dH); 0: accept every    */
                                   /* proposal (molecular-dynamics trajectories for  */
                                   /* thermalisation; dH is still computed)          */
    int chrono;                    /* force-solve starting vectors within a          */
                                   /* trajectory: 0 zero; 1 the previous MD step's   */
                                   /* solution; 2 the linear extrapolation 2x1 - x2  */
                                   /* of the last two (the first solves from zero /  */
                                   /* the previous one).  With 1 or 2 the MD is      */
                                   /* reversible to the force-solve tolerance only   */
} wd_hmc_params;

typedef struct {
    double dH;        /* H_new - H_old (FP64 sums)                                   */
    double exp_mdH;   /* exp(-dH)                                                    */
    double plaquette; /* average plaquette of the field returned                     */
    double H_old, H_new;
    double u;         /* Metropolis uniform; accepted iff u < exp(-dH)              */
    double seconds;
    int accepted;
    int cg_iters;     /* CG iterations of all force solves and the final solve      */
    int status;       /* wd_status of the trajectory                                */
} wd_hmc_result;

/* Defaults: beta 5.6, kappa 0.156, tau 1, 50 steps, seed 1, traj 0; force
 * solves FP16-sloppy to 1e-8, final solve FP64 to 1e-10; Metropolis on.
 * h: host pointer. */
void wd_hmc_defaults(wd_hmc_params *h);

/* The refresh draws of a trajectory: momenta P [V][4][3][3] (Hermitian
 * traceless, p = sum_a xi_a lambda_a / sqrt 2, xi ~ N(0,1)) and the even-site
 * Gaussian chi [Vh][4][3] (Re, Im ~ N(0, 1/2)), from Philox4x32-10 keyed by
 * seed with counter (link or site, traj, stream tag, j).  Device pointers. */
wd_status wd_hmc_draw(wd_ctx *c, double *P, double *chi, uint64_t seed, uint32_t traj);

/* MD force (Sec. 3 kernels 2 and 3) of the even-odd action at gauge field U
 * ([V][4][3][3], device) and pseudofermion phi ([Vh][4][3] even sites,
 * device): F = F_g + F_f written to F ([V][4][3][3] Hermitian traceless,
 * device), defined by dS/dt = sum tr(X F) for U -> exp(i t X) U, so that
 * dp/dt = -F.  The solve X_e = (Mhat^dag Mhat)^-1 phi_e uses p (eo = 1;
 * NULL = defaults); *cg_iters (host, may be NULL) receives its iterations.
 * Loads U as the context's gauge field. */
wd_status wd_md_force(wd_ctx *c, double *F, const double *U, const double *phi, double kappa,
                      double beta, const wd_solver_params *p, int *cg_iters);

/* One HMC trajectory (Sec. 3 steps 1-3): draw p and chi (wd_hmc_draw),
 * phi_e = Mhat^dag chi_e, H_old = 1/2 sum tr p^2 + S_g + chi^dag chi,
 * leapfrog P-Q-P with U <- exp(i dtau p) U and p <- p - dtau F, H_new with a
 * final solve, Metropolis with u from Philox (0, traj, 'M', 0) (or accept
 * without the test when h->metropolis is 0).  U
 * ([V][4][3][3], device) is replaced by the proposal when accepted and left
 * unchanged otherwise; the context's packed links follow U either way.
 * h, r: host pointers.  A failed solve rejects and returns its status. */
wd_status hmc_trajectory(wd_ctx *c, double *U, const wd_hmc_params *h, wd_hmc_result *r);

/* ---------------------------------------------------------------------- */
/* Measurements on a configuration (Sec. 3: the program measures on the     */
/* gauge configuration at the end of each trajectory; the observables are   */
/* not named there -- reading: plaquette, Polyakov loop, pion correlator).   */
/* ---------------------------------------------------------------------- */

/* Average plaquette (1/(6V)) sum_{x, mu<nu} (1/3) Re tr U_munu(x) of the
 * field U ([V][4][3][3], device); *plaq: HOST.  FP64, fixed-order sums. */
wd_status wd_plaquette(wd_ctx *c, const double *U, double *plaq);

/* Polyakov loop (1/V3) sum_x (1/3) tr prod_{t=0}^{Lt-1} U_t(x, t) of the
 * field U ([V][4][3][3], device; need not be the loaded one).  out: HOST
 * [2] = {Re, Im}. */
wd_status wd_polyakov(wd_ctx *c, const double *U, double *out);

/* Point-source propagator of the loaded gauge field: column j = 3*spin +
 * colour of psi ([12][V][4][3], device, full lattice) solves M psi_j = b_j,
 * b_j = 1 at (src, spin, colour) and 0 elsewhere.  src: HOST int32[4]
 * (x,y,z,t).  The 12 columns are one batched even-odd solve with parameters
 * p (eo must be 1; NULL = defaults): Mhat^dag Mhat psi_e = Mhat^dag (b_e +
 * kappa D_eo b_o), then psi_o = b_o + kappa D_oe psi_e; p->tol bounds the
 * true residual of that normal equation.  st: HOST [12] or NULL.  Returns
 * WD_ERR_NOCONV / WD_ERR_NAN as wd_cg_solve (psi then holds the best
 * iterate); WD_ERR_ARG for a source outside the lattice. */
wd_status wd_point_propagator(wd_ctx *c, double *psi, const int32_t src[4], double kappa,
                              const wd_solver_params *p, wd_solver_stats *st);

/* Pion (pseudoscalar, zero momentum) correlator of a point-source
 * propagator psi ([12][V][4][3], device):  corr[dt] = sum over spatial x and
 * all 144 spin-colour entries of |psi(x, (src_t + dt) mod Lt)|^2, i.e.
 * tr S S^dag by gamma_5-hermiticity.  corr: HOST [Lt]; FP64 sums in a fixed
 * order. */
wd_status wd_pion_correlator(wd_ctx *c, double *corr, const double *psi, const int32_t src[4]);

/* Index tables computed on the HOST from the definition above: nb [V][8]
 * (x+mu, x-mu for mu = 0..3), cb [V], par [V].  HOST pointers. */
wd_status wd_index_tables(const int32_t dims[4], int32_t *nb, int32_t *cb, uint8_t *par);

/* The same tables as computed by the device index arithmetic the kernels use
 * (DEVICE pointers, same shapes). */
wd_status wd_debug_device_tables(wd_ctx *c, int32_t *nb, int32_t *cb, uint8_t *par);

/* Device bytes a context needs for the gauge field plus a solve of nrhs
 * right-hand sides with these parameters (p may be NULL for defaults). */
size_t wd_bytes_required(const int32_t dims[4], int nrhs, const wd_solver_params *p);

/* Per-kernel timing with HIP events on the context's stream.  When enabled,
 * every stencil launch is bracketed by events; wd_timing_read returns the
 * summed milliseconds, launch count and algorithmic bytes of the stencil
 * launches since the last reset (host pointers). */
wd_status wd_timing_enable(wd_ctx *c, int on);
wd_status wd_timing_read(wd_ctx *c, double *total_ms, int64_t *launches, double *bytes);

/* Per-kernel breakdown of the same timed launches, without resetting them:
 * one line per stencil instance, "name;launches;total_ms;algorithmic_bytes\n",
 * written to the HOST buffer buf of len bytes (WD_ERR_ARG if too small).
 * The name is the kernel's template instance as profilers print it. */
wd_status wd_timing_report(wd_ctx *c, char *buf, size_t len);

/* Autotune the launch shapes of the even-odd solver's four stencil sweeps for
 * nrhs right-hand sides in precision prec (wd_prec, | WD_LINKS_F16).  Every
 * supported shape (threads per work-group, RHS per lane, lanes per site, XCD
 * tile order, and where they apply the LDS-staged and the t-walking
 * kernels, see wd_dslash_shaped) is timed with HIP events on synthetic
 * fields, then the fastest with a cap of 2..8 work-groups per compute unit
 * (not for an LDS-staged shape), and the fastest of those, where it applies
 * (FP32 or FP16 spinors with FP32 12- or 8-real links, FP64 spinors with
 * FP64 12-real links, the register-tiled kernel, one lane per site, 1 or 2
 * RHS per lane), with its links loaded
 * non-temporally (report field lnt); a shape whose
 * vectors or norm partials are not bitwise identical to the reference shape
 * is rejected.  The fastest shapes are kept in the context and used by
 * solves with wd_solver_params.tuned = 1.  report: HOST buffer of len bytes
 * receiving one line per sweep (may be NULL).  Needs a loaded gauge field.
 * If the environment variable WD_TUNE_CACHE names a file, a shape found there
 * for the same lattice, nrhs and formats is run once against the reference
 * shape on the same synthetic inputs and adopted without a search only if its
 * vectors and norm partials agree bit for bit (report source=cache-verified,
 * candidates=1); otherwise it is reported as source=cache-rejected and the
 * sweep is tuned from scratch (source=timed).  New results are appended to
 * the file. */
wd_status wd_tune(wd_ctx *c, int nrhs, int prec, char *report, size_t len);

/* Stencil micro-benchmark: `iters` back-to-back sweeps of the stencil with
 * epilogue epi (0 plain D_oe, 1 xpay+norm D_eo, 2 fused CG residual update
 * on D_eo^dag as the solver's fourth sweep runs it: Ap = x + coef D^dag in,
 * r -= alpha Ap, |r|^2) on
 * nrhs synthetic fields of precision prec, with the tuned shape if tuned = 1
 * and one was kept, else the default.  The sweeps rotate over copies of the
 * links and fields (at least 2 GiB in all), so that they do not run from the
 * last-level cache.  *ms (HOST) receives the HIP-event time per sweep,
 * *bytes (HOST, may be NULL) its algorithmic bytes. */
wd_status wd_bench_dslash(wd_ctx *c, int nrhs, int prec, int epi, int iters, int tuned,
                          double *ms, double *bytes);

/* Faces of a lattice cut along t (the paper's next step, Sec. 4 end: running
 * over several GPUs).  For one sweep of the hopping term with output parity
 * out_parity (WD_EVEN or WD_ODD; D_eo or D_oe, H^dag if dagger), a GPU that
 * holds slices 0..Lt-1 of a t-decomposed lattice sends its neighbours
 *   forward face:  (1 -+ g_t) psi on the input sites of slice 0,
 *   backward face: U_t^dag (1 +- g_t) psi on the input sites of slice Lt-1,
 * each as the two independent spin rows of the projection (half a spinor;
 * the backward one colour-rotated by the sender), and adds the faces it
 * receives into its output sites on slices Lt-1 and 0.  On one GPU the
 * lattice wraps onto itself, so the faces packed from psi are the ones
 * received.  wd_faces_apply packs the faces of in (DEVICE, canonical parity
 * field [Vh][4][3] complex128 of the input parity, cb order) in the spinor
 * format of prec (WD_F64, WD_F32 or WD_F16, | WD_LINKS_F16 / _R18), then
 * writes to out (DEVICE, same layout, output parity) the face terms alone:
 * the t-neighbour terms across the cut on slices Lt-1 and 0, zero on every
 * other site.  Needs a loaded gauge field; WD_ERR_ARG for WD_FULL, WD_I16
 * or a bad code. */
wd_status wd_faces_apply(wd_ctx *c, double *out, const double *in, int out_parity, int dagger, int prec);

/* Face micro-benchmark on the context's lattice: `iters` packs of both faces,
 * then `iters` face updates, in the spinor format of prec; *pack_ms and
 * *apply_ms (HOST) receive the HIP-event time of one, *pack_bytes and
 * *apply_bytes (HOST, may be NULL) the bytes one must move (spinor slices,
 * links and faces, each once). */
wd_status wd_bench_faces(wd_ctx *c, int prec, int iters, double *pack_ms, double *apply_ms,
                         double *pack_bytes, double *apply_bytes);

/* Message of the last failed call on this thread (never NULL). */
const char *wd_last_error(void);

/* Library version string. */
const char *wd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WD_H */
