/*
 * wdref.c -- plain FP64 CPU oracle for two-flavour Wilson-fermion HMC.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * path.  Every routine is written for a reader who checks it against the paper
 * (arXiv:1207.2223, "Hybrid Monte Carlo with Wilson Dirac operator on the Fermi
 * GPU"), not for speed: full 4x4 gamma matrices, full 3x3 links, the even-odd
 * blocks taken as restrictions of the full operator.
 *
 * Conventions (the paper leaves them open; the readings taken are these):
 *   lattice   dims (Lx,Ly,Lz,Lt), all even; lex = x + Lx*(y + Ly*(z + Lz*t));
 *             parity = (x+y+z+t) & 1; checkerboard index cb = lex >> 1;
 *             periodic in all four directions (Sec. 1 lattice, Sec. 3
 *             neighbour routine).
 *   spinor    psi[lex][spin 4][colour 3], complex128 (Sec. 3: N_c x 4 x N_site).
 *   links     U[lex][mu][a][b] = U_mu(x), the transporter from x to x+mu
 *             (Sec. 1, eq. 1 context); momenta and forces share that layout as
 *             3x3 Hermitian traceless matrices.
 *   gamma     Euclidean Hermitian chiral (DeGrand-Rossi) basis, gamma_1..4 for
 *             x,y,z,t (Sec. 3: four constant 4x4 matrices).
 *   operator  M = 1 - kappa*H with
 *             (H psi)(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu)
 *                                + (1+g_mu) U_mu(x-mu)^dag psi(x-mu),
 *             the kappa-normalised form of M = D + m (eq. 4); M^dag = 1-kappa*H^dag
 *             where H^dag swaps (1-g) and (1+g).
 *   even-odd  D_eo = even<-odd block of H, D_oe = odd<-even block;
 *             Mhat = 1 - kappa^2 D_eo D_oe on even sites.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Lattice geometry (Sec. 1: N_site points ordered in some fashion).         */
/* ------------------------------------------------------------------------ */

static long vol(const int32_t d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static long lex_of(const int32_t d[4], const int x[4])
{
    return x[0] + (long)d[0] * (x[1] + (long)d[1] * (x[2] + (long)d[2] * x[3]));
}

static void coords_of(const int32_t d[4], long lex, int x[4])
{
    for (int mu = 0; mu < 4; mu++) {
        x[mu] = (int)(lex % d[mu]);
        lex /= d[mu];
    }
}

static int parity_of(const int32_t d[4], long lex)
{
    int x[4];
    coords_of(d, lex, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* Neighbour index computed from the coordinates (Sec. 3: the neighbour
 * indices are computed, not stored).  dir = +1 or -1, periodic wrap. */
static long step(const int32_t d[4], long lex, int mu, int dir)
{
    int x[4];
    coords_of(d, lex, x);
    x[mu] = (x[mu] + dir + d[mu]) % d[mu];
    return lex_of(d, x);
}

int wdref_check_dims(const int32_t d[4])
{
    for (int mu = 0; mu < 4; mu++)
        if (d[mu] < 2 || (d[mu] & 1)) return -2;
    return 0;
}

/* Index tables: nb[lex][2mu] = x+mu, nb[lex][2mu+1] = x-mu; cb[lex] = lex>>1;
 * par[lex] = parity.  eo_lex[P*Vh + cb] = lex of the cb-th site of parity P. */
int wdref_index_tables(const int32_t d[4], int32_t *nb, int32_t *cb, uint8_t *par,
                       int32_t *eo_lex)
{
    if (wdref_check_dims(d)) return -2;
    long V = vol(d), Vh = V / 2;
    for (long s = 0; s < V; s++) {
        for (int mu = 0; mu < 4; mu++) {
            nb[s * 8 + 2 * mu] = (int32_t)step(d, s, mu, +1);
            nb[s * 8 + 2 * mu + 1] = (int32_t)step(d, s, mu, -1);
        }
        cb[s] = (int32_t)(s >> 1);
        par[s] = (uint8_t)parity_of(d, s);
        if (eo_lex) eo_lex[par[s] * Vh + (s >> 1)] = (int32_t)s;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gamma matrices (Sec. 3: four constant 4x4 matrices, 8 non-zero entries in */
/* each 1 +- gamma).  Chiral basis; index 4 is gamma_5 = g1 g2 g3 g4.        */
/* ------------------------------------------------------------------------ */

static cplx G[5][4][4];
static int G_ready = 0;

static void gamma_init(void)
{
    if (G_ready) return;
    memset(G, 0, sizeof(G));
    const cplx J = _Complex_I; /* imaginary unit */
    /* gamma_1 (x) */
    G[0][0][3] = J;  G[0][1][2] = J;  G[0][2][1] = -J; G[0][3][0] = -J;
    /* gamma_2 (y) */
    G[1][0][3] = -1; G[1][1][2] = 1;  G[1][2][1] = 1;  G[1][3][0] = -1;
    /* gamma_3 (z) */
    G[2][0][2] = J;  G[2][1][3] = -J; G[2][2][0] = -J; G[2][3][1] = J;
    /* gamma_4 (t) */
    G[3][0][2] = 1;  G[3][1][3] = 1;  G[3][2][0] = 1;  G[3][3][1] = 1;
    /* gamma_5 = g1 g2 g3 g4 as a product, not typed in */
    cplx a[4][4], b[4][4];
    memcpy(a, G[0], sizeof(a));
    for (int k = 1; k < 4; k++) {
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int l = 0; l < 4; l++) s += a[i][l] * G[k][l][j];
                b[i][j] = s;
            }
        memcpy(a, b, sizeof(a));
    }
    memcpy(G[4], a, sizeof(a));
    G_ready = 1;
}

void wdref_gamma(int mu, double *out /* [4][4][2] */)
{
    gamma_init();
    memcpy(out, G[mu], sizeof(G[mu]));
}

/* ------------------------------------------------------------------------ */
/* Hopping term H and the Wilson operator M = 1 - kappa H (eq. 4, Sec. 2).   */
/* ------------------------------------------------------------------------ */

/* out(x) = sum_mu (1 - sg g_mu) U_mu(x) in(x+mu) + (1 + sg g_mu) U_mu(x-mu)^dag in(x-mu)
 * with sg = +1 for H and -1 for H^dag.  Only sites whose parity equals
 * `only_par` are written when only_par >= 0; the rest of out is untouched. */
static void hop(const int32_t d[4], const cplx *U, const cplx *in, cplx *out, int dagger,
                int only_par)
{
    gamma_init();
    long V = vol(d);
    double sg = dagger ? -1.0 : 1.0;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++) {
        if (only_par >= 0 && parity_of(d, x) != only_par) continue;
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; mu++) {
            long xf = step(d, x, mu, +1), xb = step(d, x, mu, -1);
            const cplx *Uf = U + (x * 4 + mu) * 9;  /* U_mu(x)    */
            const cplx *Ub = U + (xb * 4 + mu) * 9; /* U_mu(x-mu) */
            cplx tf[4][3], tb[4][3];
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++) {
                    cplx f = 0, g = 0;
                    for (int b = 0; b < 3; b++) {
                        f += Uf[a * 3 + b] * in[xf * 12 + s * 3 + b];
                        g += conj(Ub[b * 3 + a]) * in[xb * 12 + s * 3 + b];
                    }
                    tf[s][a] = f;
                    tb[s][a] = g;
                }
            for (int s = 0; s < 4; s++)
                for (int a = 0; a < 3; a++) {
                    cplx gf = 0, gb = 0;
                    for (int t = 0; t < 4; t++) {
                        gf += G[mu][s][t] * tf[t][a];
                        gb += G[mu][s][t] * tb[t][a];
                    }
                    acc[s][a] += (tf[s][a] - sg * gf) + (tb[s][a] + sg * gb);
                }
        }
        memcpy(out + x * 12, acc, sizeof(acc));
    }
}

void wdref_hop(const int32_t d[4], const double *U, const double *in, double *out, int dagger)
{
    hop(d, (const cplx *)U, (const cplx *)in, (cplx *)out, dagger, -1);
}

/* out = in - kappa * H in   (M), or with H^dag (M^dag) */
static void wilson(const int32_t d[4], const cplx *U, double kappa, const cplx *in, cplx *out,
                   int dagger)
{
    long n = vol(d) * 12;
    hop(d, U, in, out, dagger, -1);
    for (long i = 0; i < n; i++) out[i] = in[i] - kappa * out[i];
}

void wdref_wilson(const int32_t d[4], const double *U, double kappa, const double *in,
                  double *out, int dagger)
{
    wilson(d, (const cplx *)U, kappa, (const cplx *)in, (cplx *)out, dagger);
}

void wdref_mdagm(const int32_t d[4], const double *U, double kappa, const double *in,
                 double *out)
{
    long n = vol(d) * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    wilson(d, (const cplx *)U, kappa, (const cplx *)in, t, 0);
    wilson(d, (const cplx *)U, kappa, t, (cplx *)out, 1);
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Even-odd blocks: D_{P, 1-P} is the restriction of H to output parity P   */
/* and input parity 1-P.  Parity fields are [Vh][4][3] in cb order.         */
/* ------------------------------------------------------------------------ */

static long *eo_table(const int32_t d[4])
{
    long V = vol(d), Vh = V / 2;
    long *t = malloc(sizeof(long) * V);
    for (long s = 0; s < V; s++) t[parity_of(d, s) * Vh + (s >> 1)] = s;
    return t;
}

/* out_par (parity P) = [H or H^dag] applied to in_par living on parity 1-P */
static void hop_block(const int32_t d[4], const cplx *U, const cplx *in_par, cplx *out_par,
                      int out_parity, int dagger)
{
    long V = vol(d), Vh = V / 2;
    long *tab = eo_table(d);
    cplx *full_in = calloc(V * 12, sizeof(cplx));
    cplx *full_out = calloc(V * 12, sizeof(cplx));
    int in_parity = 1 - out_parity;
    for (long i = 0; i < Vh; i++)
        memcpy(full_in + tab[in_parity * Vh + i] * 12, in_par + i * 12, 12 * sizeof(cplx));
    hop(d, U, full_in, full_out, dagger, out_parity);
    for (long i = 0; i < Vh; i++)
        memcpy(out_par + i * 12, full_out + tab[out_parity * Vh + i] * 12, 12 * sizeof(cplx));
    free(full_in);
    free(full_out);
    free(tab);
}

void wdref_hop_eo(const int32_t d[4], const double *U, const double *in_par, double *out_par,
                  int out_parity, int dagger)
{
    hop_block(d, (const cplx *)U, (const cplx *)in_par, (cplx *)out_par, out_parity, dagger);
}

/* Mhat = 1 - kappa^2 D_eo D_oe (dagger: 1 - kappa^2 (H^dag)_eo (H^dag)_oe) */
static void mhat(const int32_t d[4], const cplx *U, double kappa, const cplx *in_e, cplx *out_e,
                 int dagger)
{
    long Vh = vol(d) / 2, n = Vh * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    hop_block(d, U, in_e, t, 1, dagger);
    hop_block(d, U, t, out_e, 0, dagger);
    for (long i = 0; i < n; i++) out_e[i] = in_e[i] - kappa * kappa * out_e[i];
    free(t);
}

void wdref_mhat(const int32_t d[4], const double *U, double kappa, const double *in_e,
                double *out_e, int dagger)
{
    mhat(d, (const cplx *)U, kappa, (const cplx *)in_e, (cplx *)out_e, dagger);
}

void wdref_mhatdag_mhat(const int32_t d[4], const double *U, double kappa, const double *in_e,
                        double *out_e)
{
    long n = vol(d) / 2 * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    mhat(d, (const cplx *)U, kappa, (const cplx *)in_e, t, 0);
    mhat(d, (const cplx *)U, kappa, t, (cplx *)out_e, 1);
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient on a Hermitian positive-definite operator (eq. 3: the  */
/* inverse applied to a vector in O(N) steps).  x0 = 0; stops when the       */
/* true residual |b - A x| / |b| <= tol, recomputed in FP64.                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const int32_t *d;
    const cplx *U;
    double kappa;
    int eo;
} op_ctx;

static void apply_A(const op_ctx *c, const cplx *in, cplx *out)
{
    if (c->eo)
        wdref_mhatdag_mhat(c->d, (const double *)c->U, c->kappa, (const double *)in,
                           (double *)out);
    else
        wdref_mdagm(c->d, (const double *)c->U, c->kappa, (const double *)in, (double *)out);
}

static double dot_re(const cplx *a, const cplx *b, long n)
{
    double s = 0;
    for (long i = 0; i < n; i++) s += creal(conj(a[i]) * b[i]);
    return s;
}

/* Returns 0 on convergence, -5 when maxiter is reached.  iters and the true
 * relative residual are written out; hist (optional, length maxiter+1) gets
 * |r_k|/|b| of the iterated residual. */
int wdref_cg(const int32_t d[4], const double *U, double kappa, int eo, const double *b_,
             double *x_, double tol, int maxiter, int *iters, double *true_rel, double *hist)
{
    op_ctx c = {d, (const cplx *)U, kappa, eo};
    long n = vol(d) * 12 / (eo ? 2 : 1);
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n);
    double bb = dot_re(b, b, n);
    int k = 0, status = -5;
    memset(x, 0, sizeof(cplx) * n);
    if (bb == 0.0) {
        *iters = 0;
        *true_rel = 0.0;
        free(r); free(p); free(Ap);
        return 0;
    }
    memcpy(r, b, sizeof(cplx) * n);
    memcpy(p, b, sizeof(cplx) * n);
    double rr = bb;
    if (hist) hist[0] = 1.0;
    while (k < maxiter) {
        apply_A(&c, p, Ap);
        double pAp = dot_re(p, Ap, n);
        double alpha = rr / pAp;
        for (long i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
        }
        double rr_new = dot_re(r, r, n);
        k++;
        if (hist) hist[k] = sqrt(rr_new / bb);
        if (rr_new <= tol * tol * bb) {
            /* confirm on the true residual; continue from it if it is not met */
            apply_A(&c, x, Ap);
            for (long i = 0; i < n; i++) r[i] = b[i] - Ap[i];
            double tr = dot_re(r, r, n);
            if (tr <= tol * tol * bb) {
                status = 0;
                rr = tr;
                break;
            }
            memcpy(p, r, sizeof(cplx) * n);
            rr = tr;
            continue;
        }
        double beta = rr_new / rr;
        rr = rr_new;
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
    }
    apply_A(&c, x, Ap);
    for (long i = 0; i < n; i++) r[i] = b[i] - Ap[i];
    *true_rel = sqrt(dot_re(r, r, n) / bb);
    *iters = k;
    free(r); free(p); free(Ap);
    return status;
}

/* ------------------------------------------------------------------------ */
/* 3x3 complex helpers for the gauge part (Sec. 2-3: gauge force, gauge      */
/* field evolution).                                                          */
/* ------------------------------------------------------------------------ */

static void mm(const cplx *a, const cplx *b, cplx *c) /* c = a b */
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[i * 3 + k] * b[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(c, t, sizeof(t));
}

static void dag(const cplx *a, cplx *c) /* c = a^dag */
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[i * 3 + j] = conj(a[j * 3 + i]);
    memcpy(c, t, sizeof(t));
}

static cplx tr3(const cplx *a) { return a[0] + a[4] + a[8]; }

static const cplx *link(const cplx *U, long x, int mu) { return U + (x * 4 + mu) * 9; }

/* Traceless Hermitian part: (W - W^dag)/(2i) with the trace removed */
static void ta_herm(const cplx *W, cplx *F)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            t[i * 3 + j] = (W[i * 3 + j] - conj(W[j * 3 + i])) / (2.0 * _Complex_I);
    cplx tr = tr3(t) / 3.0;
    for (int i = 0; i < 3; i++) t[i * 4] -= tr;
    memcpy(F, t, sizeof(t));
}

/* Plaquette U_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
static void plaq(const int32_t d[4], const cplx *U, long x, int mu, int nu, cplx *P)
{
    cplx a[9], b[9];
    long xm = step(d, x, mu, +1), xn = step(d, x, nu, +1);
    mm(link(U, x, mu), link(U, xm, nu), a);
    dag(link(U, xn, mu), b);
    mm(a, b, a);
    dag(link(U, x, nu), b);
    mm(a, b, P);
}

/* Average plaquette (1/6V) sum_{x, mu<nu} Re tr U_munu / 3 */
double wdref_plaquette(const int32_t d[4], const double *U_)
{
    const cplx *U = (const cplx *)U_;
    long V = vol(d);
    double s = 0;
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                cplx P[9];
                plaq(d, U, x, mu, nu, P);
                s += creal(tr3(P)) / 3.0;
            }
    return s / (6.0 * V);
}

/* Wilson plaquette action S_g = beta sum_{x, mu<nu} (1 - Re tr U_munu / 3) */
double wdref_gauge_action(const int32_t d[4], const double *U_, double beta)
{
    return beta * 6.0 * vol(d) * (1.0 - wdref_plaquette(d, U_));
}

/* Gauge force F_g(x,mu) = (beta/3) TA[U_mu(x) A_mu(x)], A = sum of the six
 * staples, defined by dS_g/dt = sum tr(X F_g) for U -> exp(i t X) U. */
void wdref_gauge_force(const int32_t d[4], const double *U_, double beta, double *F_)
{
    const cplx *U = (const cplx *)U_;
    cplx *F = (cplx *)F_;
    long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++) {
            cplx A[9] = {0}, a[9], b[9];
            for (int nu = 0; nu < 4; nu++) {
                if (nu == mu) continue;
                long xm = step(d, x, mu, +1), xn = step(d, x, nu, +1);
                long xmn = step(d, xm, nu, -1), xbn = step(d, x, nu, -1);
                /* upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
                dag(link(U, xn, mu), a);
                mm(link(U, xm, nu), a, a);
                dag(link(U, x, nu), b);
                mm(a, b, a);
                for (int i = 0; i < 9; i++) A[i] += a[i];
                /* lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) */
                dag(link(U, xmn, nu), a);
                dag(link(U, xbn, mu), b);
                mm(a, b, a);
                mm(a, link(U, xbn, nu), a);
                for (int i = 0; i < 9; i++) A[i] += a[i];
            }
            cplx W[9];
            mm(link(U, x, mu), A, W);
            cplx Fl[9];
            ta_herm(W, Fl);
            for (int i = 0; i < 9; i++) F[(x * 4 + mu) * 9 + i] = (beta / 3.0) * Fl[i];
        }
}

/* Fermion force from the spinor pair (X, Y) (Sec. 3: driving force due to the
 * fermion fields, with its gamma_mu products).  Per link:
 *   Z = U_mu(x) sum_s [(1-g_mu) X(x+mu)]_s Y(x)_s^dag
 *       - sum_s [(1+g_mu) X(x)]_s Y(x+mu)_s^dag U_mu(x)^dag
 *   F = coef * TA[Z],   coef = -2 kappa (full) or -2 kappa^2 (even-odd),
 * which follows from dS_f/dt = coef' Re(Y^dag dH/dt X). */
static void fermion_force_xy(const int32_t d[4], const cplx *U, const cplx *X, const cplx *Y,
                             double coef, cplx *F)
{
    gamma_init();
    long V = vol(d);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++) {
            long xf = step(d, x, mu, +1);
            cplx P[9] = {0}, Q[9] = {0};
            for (int s = 0; s < 4; s++) {
                cplx pm[3], pp[3];
                for (int a = 0; a < 3; a++) {
                    cplx gm = 0, gp = 0;
                    for (int t = 0; t < 4; t++) {
                        gm += G[mu][s][t] * X[xf * 12 + t * 3 + a];
                        gp += G[mu][s][t] * X[x * 12 + t * 3 + a];
                    }
                    pm[a] = X[xf * 12 + s * 3 + a] - gm; /* [(1-g) X(x+mu)]_s */
                    pp[a] = X[x * 12 + s * 3 + a] + gp;  /* [(1+g) X(x)]_s    */
                }
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) {
                        P[a * 3 + b] += pm[a] * conj(Y[x * 12 + s * 3 + b]);
                        Q[a * 3 + b] += pp[a] * conj(Y[xf * 12 + s * 3 + b]);
                    }
            }
            cplx Z[9], t[9];
            mm(link(U, x, mu), P, Z);
            dag(link(U, x, mu), t);
            mm(Q, t, t);
            for (int i = 0; i < 9; i++) Z[i] -= t[i];
            cplx Fl[9];
            ta_herm(Z, Fl);
            for (int i = 0; i < 9; i++) F[(x * 4 + mu) * 9 + i] = coef * Fl[i];
        }
}

void wdref_fermion_force_xy(const int32_t d[4], const double *U, const double *X,
                            const double *Y, double coef, double *F)
{
    fermion_force_xy(d, (const cplx *)U, (const cplx *)X, (const cplx *)Y, coef, (cplx *)F);
}

/* Fermion force of S_f = phi^dag (A)^-1 phi with A = M^dag M (eo = 0, phi on
 * the full lattice) or Mhat^dag Mhat (eo = 1, phi on even sites).  The solve
 * runs to `tol`.  X = A^-1 phi, Y = M X (or Mhat X), then the full-lattice
 * pair is completed with X_o = D_oe X_e and Y_o = (H^dag)_oe Y_e. */
int wdref_fermion_force(const int32_t d[4], const double *U_, double kappa, int eo,
                        const double *phi, double tol, int maxiter, double *F_, int *iters)
{
    const cplx *U = (const cplx *)U_;
    long V = vol(d), Vh = V / 2, n = V * 12 / (eo ? 2 : 1);
    cplx *X = calloc(V * 12, sizeof(cplx)), *Y = calloc(V * 12, sizeof(cplx));
    cplx *sol = malloc(sizeof(cplx) * n);
    double tr;
    int st = wdref_cg(d, U_, kappa, eo, phi, (double *)sol, tol, maxiter, iters, &tr, NULL);
    if (!eo) {
        memcpy(X, sol, sizeof(cplx) * n);
        wilson(d, U, kappa, X, Y, 0);
        fermion_force_xy(d, U, X, Y, -2.0 * kappa, (cplx *)F_);
    } else {
        long *tab = eo_table(d);
        cplx *Ye = malloc(sizeof(cplx) * Vh * 12), *Xo = malloc(sizeof(cplx) * Vh * 12);
        cplx *Yo = malloc(sizeof(cplx) * Vh * 12);
        mhat(d, U, kappa, sol, Ye, 0);
        hop_block(d, U, sol, Xo, 1, 0);
        hop_block(d, U, Ye, Yo, 1, 1);
        for (long i = 0; i < Vh; i++) {
            memcpy(X + tab[i] * 12, sol + i * 12, 12 * sizeof(cplx));
            memcpy(X + tab[Vh + i] * 12, Xo + i * 12, 12 * sizeof(cplx));
            memcpy(Y + tab[i] * 12, Ye + i * 12, 12 * sizeof(cplx));
            memcpy(Y + tab[Vh + i] * 12, Yo + i * 12, 12 * sizeof(cplx));
        }
        fermion_force_xy(d, U, X, Y, -2.0 * kappa * kappa, (cplx *)F_);
        free(Ye); free(Xo); free(Yo); free(tab);
    }
    free(X); free(Y); free(sol);
    return st;
}

/* Fermion action phi^dag A^-1 phi by a solve to `tol`. */
double wdref_fermion_action(const int32_t d[4], const double *U, double kappa, int eo,
                            const double *phi_, double tol, int maxiter, int *iters)
{
    long n = vol(d) * 12 / (eo ? 2 : 1);
    cplx *X = malloc(sizeof(cplx) * n);
    double tr;
    wdref_cg(d, U, kappa, eo, phi_, (double *)X, tol, maxiter, iters, &tr, NULL);
    double s = dot_re((const cplx *)phi_, X, n);
    free(X);
    return s;
}

/* exp(i a P) for Hermitian P by its power series, summed until the terms stop
 * changing the result (Sec. 2: U and exp(ip) are conjugate; gauge evolution). */
static void expi(const cplx *P, double a, cplx *E)
{
    cplx term[9], t[9];
    memset(E, 0, sizeof(cplx) * 9);
    memset(term, 0, sizeof(term));
    for (int i = 0; i < 3; i++) E[i * 4] = term[i * 4] = 1.0;
    for (int k = 1; k < 200; k++) {
        mm(term, P, t);
        double mx = 0;
        for (int i = 0; i < 9; i++) {
            term[i] = t[i] * (_Complex_I * a / k);
            E[i] += term[i];
            if (cabs(term[i]) > mx) mx = cabs(term[i]);
        }
        if (mx < 1e-30) break;
    }
}

void wdref_expi(const double *P, double a, double *E) { expi((const cplx *)P, a, (cplx *)E); }

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* SC'11), 53-bit uniforms and the Box-Muller transform.                     */
/* ------------------------------------------------------------------------ */

void wdref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A uniform in (0,1) from 64 random bits: the top 53 bits, centred. */
static double u53(uint32_t hi, uint32_t lo)
{
    uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)v + 0.5) * (1.0 / 9007199254740992.0);
}

/* Two standard normals from one Philox block: stream tag, counter j. */
static void normal_pair(uint64_t seed, uint32_t site, uint32_t traj, uint32_t tag, uint32_t j,
                        double *n1, double *n2)
{
    uint32_t ctr[4] = {site, traj, tag, j}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    wdref_philox4x32_10(ctr, key, r);
    double u1 = u53(r[0], r[1]), u2 = u53(r[2], r[3]);
    double rad = sqrt(-2.0 * log(u1)), th = 2.0 * M_PI * u2;
    *n1 = rad * cos(th);
    *n2 = rad * sin(th);
}

void wdref_normal_pair(uint64_t seed, uint32_t site, uint32_t traj, uint32_t tag, uint32_t j,
                       double *out2)
{
    normal_pair(seed, site, traj, tag, j, out2, out2 + 1);
}

double wdref_uniform(uint64_t seed, uint32_t site, uint32_t traj, uint32_t tag, uint32_t j)
{
    uint32_t ctr[4] = {site, traj, tag, j}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    wdref_philox4x32_10(ctr, key, r);
    return u53(r[0], r[1]);
}

#define TAG_MOM 0x50u  /* momenta       */
#define TAG_CHI 0x43u  /* pseudofermion */
#define TAG_MET 0x4Du  /* Metropolis    */

/* Momenta p(x,mu) = sum_a xi_a lambda_a / sqrt(2), xi ~ N(0,1), so that the
 * density is exp(-tr p^2 / 2) (eq. 5 kinetic term).  Gell-Mann matrices are
 * built entry by entry here. */
void wdref_draw_momenta(const int32_t d[4], uint64_t seed, uint32_t traj, double *P_)
{
    cplx *P = (cplx *)P_;
    long V = vol(d);
    const double r3 = 1.0 / sqrt(3.0);
    for (long x = 0; x < V; x++)
        for (int mu = 0; mu < 4; mu++) {
            double xi[8];
            for (int j = 0; j < 4; j++)
                normal_pair(seed, (uint32_t)(x * 4 + mu), traj, TAG_MOM, (uint32_t)j,
                            &xi[2 * j], &xi[2 * j + 1]);
            cplx m[9] = {0};
            const cplx J = _Complex_I; /* imaginary unit */
            /* sum_a xi_a lambda_a */
            m[0 * 3 + 1] += xi[0]; m[1 * 3 + 0] += xi[0];          /* lambda_1 */
            m[0 * 3 + 1] += -J * xi[1]; m[1 * 3 + 0] += J * xi[1];  /* lambda_2 */
            m[0] += xi[2]; m[4] -= xi[2];                           /* lambda_3 */
            m[0 * 3 + 2] += xi[3]; m[2 * 3 + 0] += xi[3];          /* lambda_4 */
            m[0 * 3 + 2] += -J * xi[4]; m[2 * 3 + 0] += J * xi[4];  /* lambda_5 */
            m[1 * 3 + 2] += xi[5]; m[2 * 3 + 1] += xi[5];          /* lambda_6 */
            m[1 * 3 + 2] += -J * xi[6]; m[2 * 3 + 1] += J * xi[6];  /* lambda_7 */
            m[0] += xi[7] * r3; m[4] += xi[7] * r3; m[8] -= 2.0 * xi[7] * r3; /* lambda_8 */
            for (int i = 0; i < 9; i++) P[(x * 4 + mu) * 9 + i] = m[i] / sqrt(2.0);
        }
}

/* chi with density exp(-chi^dag chi): Re, Im ~ N(0, 1/2) (Sec. 2: chi drawn
 * from a Gaussian).  nsites = Vh for even-odd (site = cb) or V (site = lex). */
void wdref_draw_chi(long nsites, uint64_t seed, uint32_t traj, double *chi_)
{
    cplx *chi = (cplx *)chi_;
    const double s = sqrt(0.5);
    for (long i = 0; i < nsites; i++)
        for (int j = 0; j < 12; j++) {
            double a, b;
            normal_pair(seed, (uint32_t)i, traj, TAG_CHI, (uint32_t)j, &a, &b);
            chi[i * 12 + j] = s * a + _Complex_I * (s * b);
        }
}

double wdref_kinetic(const int32_t d[4], const double *P_)
{
    const cplx *P = (const cplx *)P_;
    long V = vol(d);
    double s = 0;
    for (long l = 0; l < V * 4; l++) {
        cplx t[9];
        mm(P + l * 9, P + l * 9, t);
        s += 0.5 * creal(tr3(t));
    }
    return s;
}

/* Total MD force F = F_g + F_f (Sec. 3, kernels 2 and 3). */
static int md_force(const int32_t d[4], const double *U, double beta, double kappa, int eo,
                    const double *phi, double tol, int maxiter, double *F, int *iters)
{
    long nl = vol(d) * 4 * 9;
    double *Ff = malloc(sizeof(cplx) * nl);
    wdref_gauge_force(d, U, beta, F);
    int st = wdref_fermion_force(d, U, kappa, eo, phi, tol, maxiter, Ff, iters);
    for (long i = 0; i < nl * 2; i++) F[i] += Ff[i];
    free(Ff);
    return st;
}

int wdref_md_force(const int32_t d[4], const double *U, double beta, double kappa, int eo,
                   const double *phi, double tol, int maxiter, double *F, int *iters)
{
    return md_force(d, U, beta, kappa, eo, phi, tol, maxiter, F, iters);
}

/* p <- p - eps F */
static void p_step(long nl, cplx *P, const cplx *F, double eps)
{
    for (long i = 0; i < nl; i++) P[i] -= eps * F[i];
}

/* U <- exp(i eps p) U */
static void u_step(long nlinks, cplx *U, const cplx *P, double eps)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nlinks; l++) {
        cplx E[9];
        expi(P + l * 9, eps, E);
        mm(E, U + l * 9, U + l * 9);
    }
}

/* Leapfrog in the P Q P order (Sec. 3, step 2): half step in p, then
 * nsteps-1 rounds of (full U, full p), a last full U and a closing half p. */
int wdref_leapfrog(const int32_t d[4], double *U_, double *P_, double beta, double kappa,
                   int eo, const double *phi, double tau, int nsteps, double tol, int maxiter,
                   int *cg_iters)
{
    cplx *U = (cplx *)U_, *P = (cplx *)P_;
    long nlinks = vol(d) * 4, nl = nlinks * 9;
    double eps = tau / nsteps;
    cplx *F = malloc(sizeof(cplx) * nl);
    int it, tot = 0, st = 0;
    st |= md_force(d, U_, beta, kappa, eo, phi, tol, maxiter, (double *)F, &it);
    tot += it;
    p_step(nl, P, F, 0.5 * eps);
    for (int k = 0; k < nsteps; k++) {
        u_step(nlinks, U, P, eps);
        st |= md_force(d, U_, beta, kappa, eo, phi, tol, maxiter, (double *)F, &it);
        tot += it;
        p_step(nl, P, F, (k == nsteps - 1) ? 0.5 * eps : eps);
    }
    free(F);
    *cg_iters = tot;
    return st;
}

/* One HMC trajectory (Sec. 2 and the three steps of Sec. 3): refresh p and
 * phi = M^dag chi, leapfrog, Metropolis on H_new - H_old.  U is replaced by
 * the proposal when accepted and left as it was otherwise.
 * out[0]=dH, out[1]=accepted, out[2]=plaquette after, out[3]=H_old,
 * out[4]=H_new, out[5]=S_f at the start by a solve (equals chi^dag chi),
 * out[6]=CG iterations of the force and final-H solves (the check solve of
 * out[5] is not counted), out[7]=Metropolis uniform. */
int wdref_hmc_trajectory(const int32_t d[4], double *U_, double beta, double kappa, int eo,
                         double tau, int nsteps, uint64_t seed, uint32_t traj, double tol_force,
                         double tol_h, int maxiter, double *out)
{
    long V = vol(d), nlinks = V * 4, nl = nlinks * 9;
    long ns = eo ? V / 2 : V, n = ns * 12;
    cplx *U0 = malloc(sizeof(cplx) * nl), *P = malloc(sizeof(cplx) * nl);
    cplx *chi = malloc(sizeof(cplx) * n), *phi = malloc(sizeof(cplx) * n);
    memcpy(U0, U_, sizeof(cplx) * nl);
    wdref_draw_momenta(d, seed, traj, (double *)P);
    wdref_draw_chi(ns, seed, traj, (double *)chi);
    if (eo)
        mhat(d, (const cplx *)U_, kappa, chi, phi, 1);
    else
        wilson(d, (const cplx *)U_, kappa, chi, phi, 1);
    int it0, it1, itf;
    double sf0 = wdref_fermion_action(d, U_, kappa, eo, (double *)phi, tol_h, maxiter, &it0);
    double h_old = wdref_kinetic(d, (double *)P) + wdref_gauge_action(d, U_, beta) +
                   dot_re(chi, chi, n);
    int st = wdref_leapfrog(d, U_, (double *)P, beta, kappa, eo, (double *)phi, tau, nsteps,
                            tol_force, maxiter, &itf);
    double sf1 = wdref_fermion_action(d, U_, kappa, eo, (double *)phi, tol_h, maxiter, &it1);
    double h_new = wdref_kinetic(d, (double *)P) + wdref_gauge_action(d, U_, beta) + sf1;
    double dH = h_new - h_old;
    double u = wdref_uniform(seed, 0, traj, TAG_MET, 0);
    int acc = (u < exp(-dH));
    if (!acc) memcpy(U_, U0, sizeof(cplx) * nl);
    out[0] = dH;
    out[1] = acc;
    out[2] = wdref_plaquette(d, U_);
    out[3] = h_old;
    out[4] = h_new;
    out[5] = sf0;
    out[6] = it1 + itf;
    (void)it0;
    out[7] = u;
    free(U0); free(P); free(chi); free(phi);
    return st;
}

/* ------------------------------------------------------------------------ */
/* End-of-trajectory measurements (Sec. 3: "at the end of each trajectory    */
/* measurements are carried out on the gauge configuration"; the paper does  */
/* not say which -- reading: Polyakov loop and the point-source pion         */
/* correlator, besides the plaquette).                                       */
/* ------------------------------------------------------------------------ */

/* Polyakov loop: (1/V3) sum over spatial sites of (1/3) tr prod_t U_t(x,t),
 * the product taken in increasing t.  out = {Re, Im}. */
void wdref_polyakov(const int32_t d[4], const double *U_, double *out)
{
    const cplx *U = (const cplx *)U_;
    const long v3 = (long)d[0] * d[1] * d[2];
    cplx sum = 0;
    for (long s = 0; s < v3; s++) {
        cplx P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, T[9];
        for (int t = 0; t < d[3]; t++) {
            mm(P, link(U, s + v3 * t, 3), T);
            memcpy(P, T, sizeof(T));
        }
        sum += tr3(P) / 3.0;
    }
    sum /= (double)v3;
    out[0] = creal(sum);
    out[1] = cimag(sum);
}

/* Point-source propagator: column j = 3*spin + colour of psi ([12][V][4][3])
 * solves M psi_j = b_j with b_j = delta(x, src) delta(spin) delta(colour), by
 * CG on the full normal equations M^dag M psi = M^dag b (the definition, no
 * even-odd split).  Returns 0 when all 12 converge to tol; iters (may be
 * NULL) gets the summed CG iterations. */
int wdref_point_propagator(const int32_t d[4], const double *U, double kappa, const int32_t src[4],
                           double tol, int maxiter, double *psi_, int *iters)
{
    const long V = vol(d), n = V * 12;
    int x0[4] = {src[0], src[1], src[2], src[3]};
    const long s0 = lex_of(d, x0);
    cplx *b = calloc(n, sizeof(cplx)), *rhs = malloc(sizeof(cplx) * n);
    int status = 0, total = 0;
    for (int j = 0; j < 12; j++) {
        memset(b, 0, sizeof(cplx) * n);
        b[s0 * 12 + j] = 1.0;
        wilson(d, (const cplx *)U, kappa, b, rhs, 1); /* M^dag b */
        int it;
        double tr;
        int st = wdref_cg(d, U, kappa, 0, (const double *)rhs, psi_ + (size_t)j * n * 2, tol, maxiter,
                          &it, &tr, NULL);
        total += it;
        if (st != 0) status = st;
    }
    if (iters) *iters = total;
    free(b);
    free(rhs);
    return status;
}

/* Pion correlator of a point-source propagator (psi as above):
 * C(dt) = sum over spatial sites x and the 12 x 12 spin-colour entries of
 * |psi_j(x, (t0 + dt) mod Lt)|^2, t0 = src time; by gamma_5-hermiticity this
 * is the zero-momentum pseudoscalar two-point function tr[S S^dag]. */
void wdref_pion_correlator(const int32_t d[4], const double *psi_, const int32_t src[4], double *corr)
{
    const cplx *psi = (const cplx *)psi_;
    const long V = vol(d), v3 = (long)d[0] * d[1] * d[2];
    for (int dt = 0; dt < d[3]; dt++) {
        const int t = (src[3] + dt) % d[3];
        double c = 0.0;
        for (int j = 0; j < 12; j++)
            for (long s = 0; s < v3; s++)
                for (int k = 0; k < 12; k++) {
                    const cplx z = psi[((size_t)j * V + s + v3 * t) * 12 + k];
                    c += creal(z) * creal(z) + cimag(z) * cimag(z);
                }
        corr[dt] = c;
    }
}
