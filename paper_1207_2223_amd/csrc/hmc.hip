// hmc.hip -- molecular-dynamics force and HMC trajectory for two-flavour
// Wilson fermions (Sec. 2 Hamiltonian eq. 5; Sec. 3 kernels 2-4: gauge force,
// fermion force with momentum update, gauge-field evolution; the three steps
// of a trajectory: refresh, leapfrog, accept/reject).
//
// Link-level fields (gauge field, momenta, forces) use the canonical layout
// [V][4][3][3] complex128, one thread per link.  The action is even-odd
// preconditioned, S_f = phi_e^dag (Mhat^dag Mhat)^-1 phi_e, with phi_e =
// Mhat^dag chi_e; the force solves go through wd_cg_solve (mixed precision
// allowed), the final-Hamiltonian solve to its own tolerance.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
// the 64-bit seed, counter (site, trajectory, stream tag, j); uniforms from
// the top 53 of 64 bits, centred; normals by Box-Muller.
//   momenta  link (x, mu): 8 normals from j = 0..3, tag 0x50,
//            p = sum_a xi_a lambda_a / sqrt(2)
//   chi      even site cb: component j (spin*3+colour) from pair j, tag 0x43,
//            Re, Im = (n1, n2) / sqrt(2)
//   accept   u from counter (0, traj, 0x4D, 0)
#include <math.h>
#include <stdio.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "wd_internal.h"

namespace wd {

namespace {

constexpr int kB = 256;
constexpr unsigned TAG_MOM = 0x50u, TAG_CHI = 0x43u, TAG_MET = 0x4Du;

__host__ __device__ inline void philox4x32_10(const uint32_t ctr[4], uint32_t k0, uint32_t k1,
                                              uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; round++) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t a = (uint64_t)0xD2511F53u * c0, b = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0, n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__host__ __device__ inline double unif53(uint32_t hi, uint32_t lo)
{
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)v + 0.5) * (1.0 / 9007199254740992.0);
}

__host__ __device__ inline void normals(uint64_t seed, uint32_t site, uint32_t traj, uint32_t tag,
                                        uint32_t j, double *n1, double *n2)
{
    const uint32_t ctr[4] = {site, traj, tag, j};
    uint32_t r[4];
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), r);
    const double u1 = unif53(r[0], r[1]), u2 = unif53(r[2], r[3]);
    const double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
    *n1 = rad * cos(th);
    *n2 = rad * sin(th);
}

// ----- 3x3 complex matrices (row-major double2) -----
struct M3 {
    double2 e[9];
};

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b)  // a * conj(b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ inline M3 load_m3(const double *p)
{
    M3 m;
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int k = 0; k < 9; k++) m.e[k] = q[k];
    return m;
}
__device__ inline void store_m3(double *p, const M3 &m)
{
    double2 *q = reinterpret_cast<double2 *>(p);
#pragma unroll
    for (int k = 0; k < 9; k++) q[k] = m.e[k];
}
__device__ inline M3 mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double2 s = cmul(a.e[3 * i], b.e[j]);
            s = cadd(s, cmul(a.e[3 * i + 1], b.e[3 + j]));
            s = cadd(s, cmul(a.e[3 * i + 2], b.e[6 + j]));
            c.e[3 * i + j] = s;
        }
    return c;
}
__device__ inline M3 dagger(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) c.e[3 * i + j] = make_double2(a.e[3 * j + i].x, -a.e[3 * j + i].y);
    return c;
}
__device__ inline M3 mul_dag(const M3 &a, const M3 &b) { return mul(a, dagger(b)); }
// traceless Hermitian part (W - W^dag)/(2i) - tr/3
__device__ inline M3 ta_herm(const M3 &w)
{
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double2 a = w.e[3 * i + j], b = w.e[3 * j + i];
            // (a - conj(b)) / (2i) = ((a.y + b.y) - i (a.x - b.x)) / 2
            f.e[3 * i + j] = make_double2(0.5 * (a.y + b.y), -0.5 * (a.x - b.x));
        }
    const double tr = (f.e[0].x + f.e[4].x + f.e[8].x) / 3.0;
    f.e[0].x -= tr;
    f.e[4].x -= tr;
    f.e[8].x -= tr;
    return f;
}

// lex <-> coordinates, periodic neighbours on the full lattice
__device__ inline void coords_lex(const Geom &g, int lex, int c[4])
{
    c[0] = lex % g.L[0];
    int r = lex / g.L[0];
    c[1] = r % g.L[1];
    r /= g.L[1];
    c[2] = r % g.L[2];
    c[3] = r / g.L[2];
}
__device__ inline int lex_of(const Geom &g, const int c[4])
{
    return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}
__device__ inline int shift(const Geom &g, const int c[4], int mu, int d)
{
    int y[4] = {c[0], c[1], c[2], c[3]};
    y[mu] += d;
    if (y[mu] == g.L[mu]) y[mu] = 0;
    if (y[mu] < 0) y[mu] = g.L[mu] - 1;
    return lex_of(g, y);
}
__device__ inline int shift2(const Geom &g, const int c[4], int mu, int d, int nu, int e)
{
    int y[4] = {c[0], c[1], c[2], c[3]};
    y[mu] = (y[mu] + d + g.L[mu]) % g.L[mu];
    y[nu] = (y[nu] + e + g.L[nu]) % g.L[nu];
    return lex_of(g, y);
}

__device__ inline const double *lk(const double *U, int x, int mu) { return U + ((size_t)x * 4 + mu) * 18; }

// ----- kernels -----

__global__ void __launch_bounds__(kB) k_draw_momenta(double *P, Geom g, uint64_t seed, uint32_t traj)
{
    const int l = blockIdx.x * kB + threadIdx.x;
    if (l >= 8 * g.Vh) return;
    double xi[8];
    for (int j = 0; j < 4; j++) normals(seed, (uint32_t)l, traj, TAG_MOM, (uint32_t)j, &xi[2 * j], &xi[2 * j + 1]);
    const double r3 = 0.5773502691896258, s = 0.7071067811865476;
    M3 m;
    m.e[0] = make_double2((xi[2] + xi[7] * r3) * s, 0);
    m.e[4] = make_double2((-xi[2] + xi[7] * r3) * s, 0);
    m.e[8] = make_double2(-2.0 * xi[7] * r3 * s, 0);
    m.e[1] = make_double2(xi[0] * s, -xi[1] * s);
    m.e[3] = make_double2(xi[0] * s, xi[1] * s);
    m.e[2] = make_double2(xi[3] * s, -xi[4] * s);
    m.e[6] = make_double2(xi[3] * s, xi[4] * s);
    m.e[5] = make_double2(xi[5] * s, -xi[6] * s);
    m.e[7] = make_double2(xi[5] * s, xi[6] * s);
    store_m3(P + (size_t)l * 18, m);
}

__global__ void __launch_bounds__(kB) k_draw_chi(double *chi, int nsites, uint64_t seed, uint32_t traj)
{
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= nsites) return;
    const double s = 0.7071067811865476;
    for (int j = 0; j < 12; j++) {
        double a, b;
        normals(seed, (uint32_t)i, traj, TAG_CHI, (uint32_t)j, &a, &b);
        chi[(size_t)i * 24 + 2 * j] = s * a;
        chi[(size_t)i * 24 + 2 * j + 1] = s * b;
    }
}

// F = (beta/3) TA[U_mu(x) A_mu(x)], A = sum of the six staples
__global__ void __launch_bounds__(kB) k_gauge_force(const double *U, double *F, Geom g, double beta)
{
    const int l = blockIdx.x * kB + threadIdx.x;
    if (l >= 8 * g.Vh) return;
    const int x = l >> 2, mu = l & 3;
    int c[4];
    coords_lex(g, x, c);
    M3 A;
    for (int k = 0; k < 9; k++) A.e[k] = make_double2(0, 0);
    const int xm = shift(g, c, mu, +1);
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        const int xn = shift(g, c, nu, +1), xbn = shift(g, c, nu, -1);
        const int xmbn = shift2(g, c, mu, +1, nu, -1);
        // upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        M3 t = mul_dag(load_m3(lk(U, xm, nu)), load_m3(lk(U, xn, mu)));
        t = mul_dag(t, load_m3(lk(U, x, nu)));
        // lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
        M3 b = mul(dagger(load_m3(lk(U, xmbn, nu))), dagger(load_m3(lk(U, xbn, mu))));
        b = mul(b, load_m3(lk(U, xbn, nu)));
        for (int k = 0; k < 9; k++) A.e[k] = cadd(A.e[k], cadd(t.e[k], b.e[k]));
    }
    M3 f = ta_herm(mul(load_m3(lk(U, x, mu)), A));
    const double sc = beta / 3.0;
    for (int k = 0; k < 9; k++) f.e[k] = make_double2(sc * f.e[k].x, sc * f.e[k].y);
    store_m3(F + (size_t)l * 18, f);
}

// [(1 + S g_mu) psi] as a full 4-spinor (v: 24 reals) from the projection rules
template <int MU, int S>
__device__ inline void spin_op(const double v[24], double out[24])
{
    double h[12];
    project<MU, S>(v, h);
#pragma unroll
    for (int k = 0; k < 24; k++) out[k] = 0.0;
    accumulate<MU, S>(out, h);
}

template <int MU>
__device__ inline void ff_link(const double *U, const double *X, const double *Y, double *F, int x, int xf,
                               double coef)
{
    double xv[24], xfv[24], yv[24], yfv[24], pm[24], pp[24];
    for (int k = 0; k < 24; k++) {
        xv[k] = X[(size_t)x * 24 + k];
        xfv[k] = X[(size_t)xf * 24 + k];
        yv[k] = Y[(size_t)x * 24 + k];
        yfv[k] = Y[(size_t)xf * 24 + k];
    }
    spin_op<MU, -1>(xfv, pm);  // (1 - g) X(x+mu)
    spin_op<MU, +1>(xv, pp);   // (1 + g) X(x)
    M3 Pm, Qp;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double2 s1 = make_double2(0, 0), s2 = make_double2(0, 0);
            for (int sp = 0; sp < 4; sp++) {
                const double2 pa = make_double2(pm[6 * sp + 2 * a], pm[6 * sp + 2 * a + 1]);
                const double2 yb = make_double2(yv[6 * sp + 2 * b], yv[6 * sp + 2 * b + 1]);
                s1 = cadd(s1, cmulc(pa, yb));
                const double2 qa = make_double2(pp[6 * sp + 2 * a], pp[6 * sp + 2 * a + 1]);
                const double2 yfb = make_double2(yfv[6 * sp + 2 * b], yfv[6 * sp + 2 * b + 1]);
                s2 = cadd(s2, cmulc(qa, yfb));
            }
            Pm.e[3 * a + b] = s1;
            Qp.e[3 * a + b] = s2;
        }
    const M3 u = load_m3(lk(U, x, MU));
    M3 Z = mul(u, Pm);
    const M3 t = mul_dag(Qp, u);
    for (int k = 0; k < 9; k++) Z.e[k] = make_double2(Z.e[k].x - t.e[k].x, Z.e[k].y - t.e[k].y);
    const M3 f = ta_herm(Z);
    double *Fl = F + ((size_t)x * 4 + MU) * 18;
    for (int k = 0; k < 9; k++) {
        Fl[2 * k] += coef * f.e[k].x;
        Fl[2 * k + 1] += coef * f.e[k].y;
    }
}

// F(x,mu) += coef TA[Z], Z = U (1-g)X(x+mu) Y(x)^dag - (1+g)X(x) Y(x+mu)^dag U^dag
__global__ void __launch_bounds__(kB) k_fermion_force(const double *U, const double *X, const double *Y,
                                                       double *F, Geom g, double coef)
{
    const int l = blockIdx.x * kB + threadIdx.x;
    if (l >= 8 * g.Vh) return;
    const int x = l >> 2, mu = l & 3;
    int c[4];
    coords_lex(g, x, c);
    const int xf = shift(g, c, mu, +1);
    switch (mu) {
    case 0: ff_link<0>(U, X, Y, F, x, xf, coef); break;
    case 1: ff_link<1>(U, X, Y, F, x, xf, coef); break;
    case 2: ff_link<2>(U, X, Y, F, x, xf, coef); break;
    default: ff_link<3>(U, X, Y, F, x, xf, coef); break;
    }
}

// P -= eps F
// x <- 2 x - xp, xp <- old x: linear extrapolation of the force solutions
__global__ void __launch_bounds__(kB) k_extrapolate(double *x, double *xp, long long n)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    const double cur = x[i];
    x[i] = 2.0 * cur - xp[i];
    xp[i] = cur;
}

__global__ void __launch_bounds__(kB) k_p_step(double *P, const double *F, long long n, double eps)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i < n) P[i] = fma(-eps, F[i], P[i]);
}

// U <- exp(i eps P) U.  exp by Taylor series of A = i eps P / 2^k (norm <=
// 1/4, 18 terms: truncation below 1e-20) and k squarings.
__global__ void __launch_bounds__(kB) k_u_step(double *U, const double *P, Geom g, double eps)
{
    const int l = blockIdx.x * kB + threadIdx.x;
    if (l >= 8 * g.Vh) return;
    M3 p = load_m3(P + (size_t)l * 18);
    double nrm = 0;
    for (int k = 0; k < 9; k++) nrm += p.e[k].x * p.e[k].x + p.e[k].y * p.e[k].y;
    nrm = sqrt(nrm) * fabs(eps);
    int sq = 0;
    double sc = eps;
    while (nrm > 0.25 && sq < 40) {
        nrm *= 0.5;
        sc *= 0.5;
        sq++;
    }
    M3 A;  // i sc P
    for (int k = 0; k < 9; k++) A.e[k] = make_double2(-sc * p.e[k].y, sc * p.e[k].x);
    M3 E, term;
    for (int k = 0; k < 9; k++) E.e[k] = term.e[k] = make_double2(0, 0);
    E.e[0] = E.e[4] = E.e[8] = term.e[0] = term.e[4] = term.e[8] = make_double2(1, 0);
    for (int n = 1; n <= 18; n++) {
        term = mul(term, A);
        const double inv = 1.0 / n;
        for (int k = 0; k < 9; k++) {
            term.e[k] = make_double2(term.e[k].x * inv, term.e[k].y * inv);
            E.e[k] = cadd(E.e[k], term.e[k]);
        }
    }
    for (int k = 0; k < sq; k++) E = mul(E, E);
    store_m3(U + (size_t)l * 18, mul(E, load_m3(U + (size_t)l * 18)));
}

// Per-16-thread partial sums of a per-thread value (fixed pairing tree).
__device__ inline void put_partial(double v, double *partial, int idx, bool live)
{
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 15) == 0 && live) partial[idx >> 4] = v;
}

// per site: sum_{mu<nu} Re tr U_munu / 3
__global__ void __launch_bounds__(kB) k_plaq(const double *U, Geom g, double *partial)
{
    const int x = blockIdx.x * kB + threadIdx.x;
    const int V = 2 * g.Vh;
    double s = 0;
    if (x < V) {
        int c[4];
        coords_lex(g, x, c);
        for (int mu = 0; mu < 4; mu++)
            for (int nu = mu + 1; nu < 4; nu++) {
                const int xm = shift(g, c, mu, +1), xn = shift(g, c, nu, +1);
                M3 t = mul(load_m3(lk(U, x, mu)), load_m3(lk(U, xm, nu)));
                t = mul_dag(t, load_m3(lk(U, xn, mu)));
                t = mul_dag(t, load_m3(lk(U, x, nu)));
                s += (t.e[0].x + t.e[4].x + t.e[8].x) / 3.0;
            }
    }
    put_partial(s, partial, x, x < V);
}

// per element: sum of a[i] * b[i] (a real dot of two double arrays)
__global__ void __launch_bounds__(kB) k_dot(const double *a, const double *b, long long n, double *partial)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    double v = (i < n) ? a[i] * b[i] : 0.0;
    put_partial(v, partial, (int)i, i < n);
}

// fixed-order sum of n partials into out[0]
__global__ void __launch_bounds__(1024) k_sum(const double *partial, int n, double *out)
{
    __shared__ double sh[1024];
    double v = 0;
    for (int w = threadIdx.x; w < n; w += 1024) v += partial[w];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// even-odd split/merge of canonical spinors: full[lex] <-> parity fields [cb]
__global__ void __launch_bounds__(kB) k_merge(const double *e, const double *o, double *full, Geom g)
{
    const int x = blockIdx.x * kB + threadIdx.x;
    if (x >= 2 * g.Vh) return;
    int c[4];
    coords_lex(g, x, c);
    const int P = (c[0] + c[1] + c[2] + c[3]) & 1;
    const double *src = (P ? o : e) + (size_t)(x >> 1) * 24;
    for (int k = 0; k < 24; k++) full[(size_t)x * 24 + k] = src[k];
}

}  // namespace

}  // namespace wd

using namespace wd;

#define HIPCHK(expr)                                                                               \
    do {                                                                                          \
        hipError_t e__ = (expr);                                                                  \
        if (e__ != hipSuccess)                                                                    \
            return set_error(WD_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__, __LINE__); \
    } while (0)

namespace {

struct HmcWs {
    double *U, *P, *F, *chi, *phi, *Xe, *Ye, *Xo, *Yo, *Xf, *Yf, *tmp, *partial, *scal, *Xp;
    size_t nl;   // doubles in a link field
    size_t ns;   // doubles in a parity spinor
};

wd_status hmc_ws(wd_ctx *c, HmcWs *w)
{
    const size_t V = (size_t)c->V, Vh = V / 2;
    w->nl = V * 4 * 18;
    w->ns = Vh * 24;
    void *p;
    auto get = [&](const char *n, size_t doubles, double **out) -> wd_status {
        WD_TRY(ws_get(c, n, doubles * sizeof(double), &p));
        *out = (double *)p;
        return WD_OK;
    };
    WD_TRY(get("hmc_U", w->nl, &w->U));
    WD_TRY(get("hmc_P", w->nl, &w->P));
    WD_TRY(get("hmc_F", w->nl, &w->F));
    WD_TRY(get("hmc_chi", w->ns, &w->chi));
    WD_TRY(get("hmc_phi", w->ns, &w->phi));
    WD_TRY(get("hmc_Xe", w->ns, &w->Xe));
    WD_TRY(get("hmc_Ye", w->ns, &w->Ye));
    WD_TRY(get("hmc_Xo", w->ns, &w->Xo));
    WD_TRY(get("hmc_Yo", w->ns, &w->Yo));
    WD_TRY(get("hmc_Xf", 2 * w->ns, &w->Xf));
    WD_TRY(get("hmc_Yf", 2 * w->ns, &w->Yf));
    WD_TRY(get("hmc_tmp", w->ns, &w->tmp));
    WD_TRY(get("hmc_Xp", w->ns, &w->Xp));  // the force solution of the step before (extrapolation)
    WD_TRY(get("hmc_partial", V * 4 * 18 / 16 + 64, &w->partial));  // largest reduction: a link field
    WD_TRY(get("hmc_scal", 16, &w->scal));
    return WD_OK;
}

inline unsigned nblk(long long n) { return (unsigned)((n + kB - 1) / kB); }

// sum over a device array of per-thread values produced by a kernel into a host double
wd_status finish_sum(wd_ctx *c, HmcWs &w, int nparts, double *host)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, c->stream, w.partial, nparts, w.scal);
    HIPCHK(hipGetLastError());
    void *hp;
    WD_TRY(pinned_get(c, 1, 64, &hp));
    HIPCHK(hipMemcpyAsync(hp, w.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *host = *(double *)hp;
    return WD_OK;
}

wd_status dot_host(wd_ctx *c, HmcWs &w, const double *a, const double *b, long long n, double *out)
{
    hipLaunchKernelGGL(k_dot, dim3(nblk(n)), dim3(kB), 0, c->stream, a, b, n, w.partial);
    HIPCHK(hipGetLastError());
    return finish_sum(c, w, (int)((n + 15) / 16), out);
}

wd_status plaquette_host(wd_ctx *c, HmcWs &w, const double *U, double *plaq)
{
    const int V = (int)c->V;
    hipLaunchKernelGGL(k_plaq, dim3(nblk(V)), dim3(kB), 0, c->stream, U, c->g, w.partial);
    HIPCHK(hipGetLastError());
    double s;
    WD_TRY(finish_sum(c, w, (V + 15) / 16, &s));
    *plaq = s / (6.0 * V);
    return WD_OK;
}

// out (even parity, canonical) = Mhat^dag in  (FP64 stencil sweeps)
wd_status mhat_dag(wd_ctx *c, const double *in_e, double *out_e, double kappa)
{
    Field A, T, B;
    WD_TRY(alloc_field(c, "hmc_fa", SP_F64, 1, 1, &A));
    WD_TRY(alloc_field(c, "hmc_ft", SP_F64, 1, 1, &T));
    WD_TRY(alloc_field(c, "hmc_fb", SP_F64, 1, 1, &B));
    double cf = -kappa * kappa;
    double *dcf;
    WD_TRY(upload_doubles(c, "hmc_coef", &cf, 1, &dcf));
    int zero = 0;
    int *act;
    WD_TRY(upload_ints(c, "hmc_act", &zero, 1, &act));
    HIPCHK(pack_spinor(in_e, A, 1, 0, c->g, c->stream));
    Sweep sw;
    sw.sp = SP_F64; sw.lk = c->lk64; sw.active = act; sw.nact = 1; sw.coef = dcf;
    sw.dag = 1;
    sw.P = 1; sw.epi = EPI_PLAIN; sw.in = A; sw.out = T;
    WD_TRY(run_sweep(c, sw, nullptr));
    sw.P = 0; sw.epi = EPI_XPAY; sw.in = T; sw.x = A; sw.out = B;
    WD_TRY(run_sweep(c, sw, nullptr));
    HIPCHK(unpack_spinor(B, out_e, 1, 0, c->g, c->stream));
    return WD_OK;
}

// one parity block of H (or H^dag) on canonical parity fields, FP64
wd_status hop_block(wd_ctx *c, const double *in, double *out, int out_par, int dag)
{
    return wd_dslash(c, out, in, out_par == 0 ? WD_EVEN : WD_ODD, dag, WD_F64);
}

// F = F_g + F_f for the context's current links (w.U canonical, packed),
// the fermion part from X_e = (Mhat^dag Mhat)^-1 phi_e.
wd_status md_force(wd_ctx *c, HmcWs &w, double beta, double kappa, const wd_solver_params *sp,
                   int *iters)
{
    const int nl = 8 * (int)c->Vh;
    hipLaunchKernelGGL(k_gauge_force, dim3(nblk(nl)), dim3(kB), 0, c->stream, w.U, w.F, c->g, beta);
    HIPCHK(hipGetLastError());
    wd_solver_stats st;
    wd_status s = wd_cg_solve(c, w.Xe, w.phi, 1, &kappa, sp, &st);
    *iters = st.iters;
    if (s != WD_OK) return s;
    // Y_e = Mhat X_e = X_e - k^2 D_eo D_oe X_e ;  X_o = D_oe X_e ;  Y_o = (H^dag)_oe Y_e
    WD_TRY(hop_block(c, w.Xe, w.Xo, 1, 0));
    WD_TRY(hop_block(c, w.Xo, w.tmp, 0, 0));
    {
        const double k2 = kappa * kappa;
        // Ye = Xe - k2 tmp : reuse k_p_step (P -= eps F) on copies
        HIPCHK(hipMemcpyAsync(w.Ye, w.Xe, w.ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_p_step, dim3(nblk((long long)w.ns)), dim3(kB), 0, c->stream, w.Ye, w.tmp,
                           (long long)w.ns, k2);
        HIPCHK(hipGetLastError());
    }
    WD_TRY(hop_block(c, w.Ye, w.Yo, 1, 1));
    hipLaunchKernelGGL(k_merge, dim3(nblk(2 * c->Vh)), dim3(kB), 0, c->stream, w.Xe, w.Xo, w.Xf, c->g);
    hipLaunchKernelGGL(k_merge, dim3(nblk(2 * c->Vh)), dim3(kB), 0, c->stream, w.Ye, w.Yo, w.Yf, c->g);
    hipLaunchKernelGGL(k_fermion_force, dim3(nblk(nl)), dim3(kB), 0, c->stream, w.U, w.Xf, w.Yf, w.F, c->g,
                       -2.0 * kappa * kappa);
    HIPCHK(hipGetLastError());
    return WD_OK;
}

wd_status reload_links(wd_ctx *c, const double *U)
{
    const uint32_t flags = (c->lk64 == LK_F64_12) ? WD_RECON_12 : WD_RECON_18;
    return wd_gauge_load(c, U, flags);
}

}  // namespace

extern "C" {

void wd_hmc_defaults(wd_hmc_params *h)
{
    if (!h) return;
    h->beta = 5.6;
    h->kappa = 0.156;
    h->tau = 1.0;
    h->nsteps = 50;
    h->seed = 1;
    h->traj = 0;
    wd_solver_defaults(&h->force_solver);
    h->force_solver.tol = 1e-8;
    h->force_solver.prec_sloppy = WD_F16;
    wd_solver_defaults(&h->h_solver);
    h->h_solver.tol = 1e-10;
    h->metropolis = 1;
    h->chrono = 0;
}

wd_status wd_plaquette(wd_ctx *c, const double *U, double *plaq)
{
    if (!c || !U || !plaq) return set_error(WD_ERR_ARG, "NULL argument");
    WD_HIP(hipSetDevice(c->device));
    HmcWs w{};  // only the reduction buffers
    void *p;
    WD_TRY(ws_get(c, "pl_partial", sizeof(double) * ((size_t)c->V / 16 + 64), &p));
    w.partial = (double *)p;
    WD_TRY(ws_get(c, "pl_scal", sizeof(double) * 16, &p));
    w.scal = (double *)p;
    return plaquette_host(c, w, U, plaq);
}

wd_status wd_hmc_draw(wd_ctx *c, double *P, double *chi, uint64_t seed, uint32_t traj)
{
    if (!c || !P || !chi) return set_error(WD_ERR_ARG, "NULL argument");
    WD_HIP(hipSetDevice(c->device));
    hipLaunchKernelGGL(k_draw_momenta, dim3(nblk(8 * c->Vh)), dim3(kB), 0, c->stream, P, c->g, seed, traj);
    hipLaunchKernelGGL(k_draw_chi, dim3(nblk(c->Vh)), dim3(kB), 0, c->stream, chi, (int)c->Vh, seed, traj);
    HIPCHK(hipGetLastError());
    return WD_OK;
}

wd_status wd_md_force(wd_ctx *c, double *F, const double *U, const double *phi, double kappa,
                      double beta, const wd_solver_params *p, int *cg_iters)
{
    if (!c || !F || !U || !phi) return set_error(WD_ERR_ARG, "NULL argument");
    if (!std::isfinite(kappa) || !std::isfinite(beta)) return set_error(WD_ERR_ARG, "non-finite parameter");
    wd_solver_params sp;
    wd_solver_defaults(&sp);
    if (p) sp = *p;
    if (!sp.eo) return set_error(WD_ERR_ARG, "the force uses the even-odd action (eo = 1)");
    sp.initial_guess = 0;  // the solve's workspace holds no caller data: x0 = 0
    WD_HIP(hipSetDevice(c->device));
    HmcWs w;
    WD_TRY(hmc_ws(c, &w));
    HIPCHK(hipMemcpyAsync(w.U, U, w.nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(w.phi, phi, w.ns * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    WD_TRY(reload_links(c, w.U));
    int it = 0;
    wd_status s = md_force(c, w, beta, kappa, &sp, &it);
    if (cg_iters) *cg_iters = it;
    if (s != WD_OK) return s;
    HIPCHK(hipMemcpyAsync(F, w.F, w.nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return WD_OK;
}

wd_status hmc_trajectory(wd_ctx *c, double *U, const wd_hmc_params *h, wd_hmc_result *r)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !U || !h || !r) return set_error(WD_ERR_ARG, "NULL argument");
    if (h->nsteps < 1 || !(h->tau > 0) || !std::isfinite(h->beta) || !std::isfinite(h->kappa))
        return set_error(WD_ERR_ARG, "bad HMC parameters");
    if (!h->force_solver.eo || !h->h_solver.eo) return set_error(WD_ERR_ARG, "HMC uses the even-odd action");
    if (h->chrono < 0 || h->chrono > 2) return set_error(WD_ERR_ARG, "chrono %d not in 0..2", h->chrono);
    WD_HIP(hipSetDevice(c->device));
    HmcWs w;
    WD_TRY(hmc_ws(c, &w));
    const hipStream_t s = c->stream;
    const int nl = 8 * (int)c->Vh;
    const double kappa = h->kappa, beta = h->beta, eps = h->tau / h->nsteps;
    int iters = 0, it;
    *r = wd_hmc_result{};

    // refresh: U copy, p, chi, phi = Mhat^dag chi
    HIPCHK(hipMemcpyAsync(w.U, U, w.nl * sizeof(double), hipMemcpyDeviceToDevice, s));
    WD_TRY(reload_links(c, w.U));
    WD_TRY(wd_hmc_draw(c, w.P, w.chi, h->seed, h->traj));
    WD_TRY(mhat_dag(c, w.chi, w.phi, kappa));

    double kin0, plaq0, chi2;
    WD_TRY(dot_host(c, w, w.P, w.P, (long long)w.nl, &kin0));  // sum |P_ij|^2 = tr P^2
    WD_TRY(plaquette_host(c, w, w.U, &plaq0));
    WD_TRY(dot_host(c, w, w.chi, w.chi, (long long)w.ns, &chi2));
    const double V = (double)c->V;
    const double h_old = 0.5 * kin0 + beta * 6.0 * V * (1.0 - plaq0) + chi2;

    // leapfrog P-Q-P.  chrono 1: each force solve starts from the previous
    // step's solution; chrono 2: from the linear extrapolation of the last
    // two; the first solve of a trajectory (and with 2 the second, from the
    // first) starts from zero.
    wd_solver_params fsp = h->force_solver;
    fsp.initial_guess = h->chrono ? 1 : 0;
    if (h->chrono) HIPCHK(hipMemsetAsync(w.Xe, 0, w.ns * sizeof(double), s));
    int nsolve = 0;
    auto guess = [&]() -> wd_status {
        if (h->chrono == 2 && nsolve == 1)
            HIPCHK(hipMemcpyAsync(w.Xp, w.Xe, w.ns * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (h->chrono == 2 && nsolve >= 2) {
            hipLaunchKernelGGL(k_extrapolate, dim3(nblk((long long)w.ns)), dim3(kB), 0, s, w.Xe, w.Xp,
                               (long long)w.ns);
            HIPCHK(hipGetLastError());
        }
        nsolve++;
        return WD_OK;
    };
    wd_status st = WD_OK;
    WD_TRY(guess());
    st = md_force(c, w, beta, kappa, &fsp, &it);
    iters += it;
    if (st == WD_OK) {
        hipLaunchKernelGGL(k_p_step, dim3(nblk((long long)w.nl)), dim3(kB), 0, s, w.P, w.F, (long long)w.nl, 0.5 * eps);
        for (int k = 0; k < h->nsteps && st == WD_OK; k++) {
            hipLaunchKernelGGL(k_u_step, dim3(nblk(nl)), dim3(kB), 0, s, w.U, w.P, c->g, eps);
            HIPCHK(hipGetLastError());
            WD_TRY(reload_links(c, w.U));
            WD_TRY(guess());
            st = md_force(c, w, beta, kappa, &fsp, &it);
            iters += it;
            if (st != WD_OK) break;
            hipLaunchKernelGGL(k_p_step, dim3(nblk((long long)w.nl)), dim3(kB), 0, s, w.P, w.F, (long long)w.nl,
                               (k == h->nsteps - 1) ? 0.5 * eps : eps);
        }
    }
    double h_new = NAN, plaq1 = NAN;
    if (st == WD_OK) {
        wd_solver_stats sst;
        st = wd_cg_solve(c, w.Xe, w.phi, 1, &kappa, &h->h_solver, &sst);
        iters += sst.iters;
        if (st == WD_OK) {
            double kin1, sf1;
            WD_TRY(dot_host(c, w, w.P, w.P, (long long)w.nl, &kin1));
            WD_TRY(plaquette_host(c, w, w.U, &plaq1));
            WD_TRY(dot_host(c, w, w.phi, w.Xe, (long long)w.ns, &sf1));
            h_new = 0.5 * kin1 + beta * 6.0 * V * (1.0 - plaq1) + sf1;
        }
    }
    const double dH = h_new - h_old;
    const uint32_t ctr[4] = {0, h->traj, TAG_MET, 0};
    uint32_t rr[4];
    philox4x32_10(ctr, (uint32_t)h->seed, (uint32_t)(h->seed >> 32), rr);
    const double u = unif53(rr[0], rr[1]);
    const bool acc = (st == WD_OK) && std::isfinite(dH) && (!h->metropolis || u < std::exp(-dH));
    if (acc) {
        HIPCHK(hipMemcpyAsync(U, w.U, w.nl * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        WD_TRY(reload_links(c, U));  // the context's links follow the caller's field
    }
    double plaq_out = acc ? plaq1 : plaq0;
    HIPCHK(hipStreamSynchronize(s));
    r->dH = dH;
    r->exp_mdH = std::exp(-dH);
    r->accepted = acc ? 1 : 0;
    r->plaquette = plaq_out;
    r->H_old = h_old;
    r->H_new = h_new;
    r->u = u;
    r->cg_iters = iters;
    r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    r->status = st;
    if (st != WD_OK) return st;
    return WD_OK;
}

}  // extern "C"
