// measure.hip -- measurements on a gauge configuration at the end of a
// trajectory (Sec. 3: after each trajectory the program measures on the
// configuration; the observables are not named there).  Built here: the
// Polyakov loop and the point-source propagator with the pion correlator;
// the plaquette comes with the HMC code.
//
// Propagator: column j = 3*spin + colour solves M psi_j = b_j, b_j a unit
// point source at `src`.  With M = [[1, -k D_eo], [-k D_oe, 1]] in even-odd
// blocks,
//   Mhat psi_e = b_e + k D_eo b_o,   psi_o = b_o + k D_oe psi_e,
// and Mhat psi_e = bhat is solved as Mhat^dag Mhat psi_e = Mhat^dag bhat by the
// batched CG (all 12 columns in one multi-RHS solve, any sloppy precision),
// Mhat^dag = 1 - k^2 D_oe^dag D_eo^dag.  Sums are FP64 in a fixed order.
#include <stdio.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "wd_internal.h"

namespace wd {

namespace {

constexpr int kB = 256;

#define HIPCHK(expr)                                                                               \
    do {                                                                                          \
        hipError_t e__ = (expr);                                                                  \
        if (e__ != hipSuccess)                                                                    \
            return set_error(WD_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e__), __FILE__, __LINE__); \
    } while (0)

inline unsigned nblk(long long n) { return (unsigned)((n + kB - 1) / kB); }

__global__ void __launch_bounds__(kB) k_fill(double *a, double v, long long n)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i < n) a[i] = v;
}

// y = a x + y
__global__ void __launch_bounds__(kB) k_axpy(double *y, const double *x, double a, long long n)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i < n) y[i] = fmaT(a, x[i], y[i]);
}

__global__ void __launch_bounds__(kB) k_scale(double *y, double a, long long n)
{
    const long long i = (long long)blockIdx.x * kB + threadIdx.x;
    if (i < n) y[i] *= a;
}

// column j of a [12][sites][4][3] parity field gets +1 at (site, spin-colour j)
__global__ void k_add_point(double *b, int site, long long col_doubles)
{
    const int j = threadIdx.x;
    if (j < 12) b[(size_t)j * col_doubles + (size_t)site * 24 + 2 * j] += 1.0;
}

// one column [sites][4][3] gets +1 at (site, spin-colour j)
__global__ void k_add_one(double *b, int site, int j)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) b[(size_t)site * 24 + 2 * j] += 1.0;
}

// full[lex] <- e[cb] or o[cb] by the parity of lex (canonical layouts)
__global__ void __launch_bounds__(kB) k_merge(const double *e, const double *o, double *full, Geom g)
{
    const int x = blockIdx.x * kB + threadIdx.x;
    if (x >= 2 * g.Vh) return;
    int r = x;
    const int c0 = r % g.L[0];
    r /= g.L[0];
    const int c1 = r % g.L[1];
    r /= g.L[1];
    const int c2 = r % g.L[2];
    const int c3 = r / g.L[2];
    const double *src = (((c0 + c1 + c2 + c3) & 1) ? o : e) + (size_t)(x >> 1) * 24;
#pragma unroll
    for (int k = 0; k < 24; k++) full[(size_t)x * 24 + k] = src[k];
}

// Fixed-order block sum of kB values (tree over shared memory).
__device__ inline double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

// partial[t * nb + b] = sum over the spatial sites [b*kB, (b+1)*kB) of time
// slice t of |psi_j|^2, all 12 columns and 12 spin-colour entries.
__global__ void __launch_bounds__(kB) k_corr_partial(const double *psi, long long V, int v3, int nb,
                                                     double *partial)
{
    __shared__ double sh[kB];
    const int b = blockIdx.x, t = blockIdx.y;
    const int s = b * kB + threadIdx.x;
    double acc = 0.0;
    if (s < v3) {
        const size_t site = (size_t)t * v3 + s;
        for (int j = 0; j < 12; j++) {
            const double *p = psi + ((size_t)j * V + site) * 24;
#pragma unroll
            for (int k = 0; k < 24; k++) acc = fmaT(p[k], p[k], acc);
        }
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(size_t)t * nb + b] = tot;
}

// out[dt] = sum_b partial[((t0 + dt) mod Lt) * nb + b], in b order
__global__ void k_corr_final(const double *partial, int nb, int Lt, int t0, double *out)
{
    const int dt = blockIdx.x * blockDim.x + threadIdx.x;
    if (dt >= Lt) return;
    const int t = (t0 + dt) % Lt;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += partial[(size_t)t * nb + b];
    out[dt] = s;
}

struct C3 {
    double2 e[9];
};

__device__ inline C3 load3(const double *p)
{
    C3 m;
#pragma unroll
    for (int k = 0; k < 9; k++) m.e[k] = make_double2(p[2 * k], p[2 * k + 1]);
    return m;
}

__device__ inline C3 mul3(const C3 &a, const C3 &b)
{
    C3 c;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double2 x = a.e[3 * i + k], y = b.e[3 * k + j];
                re = fmaT(x.x, y.x, re);
                re = fmaT(-x.y, y.y, re);
                im = fmaT(x.x, y.y, im);
                im = fmaT(x.y, y.x, im);
            }
            c.e[3 * i + j] = make_double2(re, im);
        }
    return c;
}

// Per spatial site s: (1/3) tr prod_{t = 0..Lt-1} U_t(s, t); block partials
// (Re, Im) in partial[2 * b + {0, 1}].
__global__ void __launch_bounds__(kB) k_poly_partial(const double *U, int v3, int Lt, double *partial)
{
    __shared__ double sh[kB];
    const int s = blockIdx.x * kB + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (s < v3) {
        C3 P = load3(U + ((size_t)s * 4 + 3) * 18);
        for (int t = 1; t < Lt; t++) P = mul3(P, load3(U + (((size_t)t * v3 + s) * 4 + 3) * 18));
        re = (P.e[0].x + P.e[4].x + P.e[8].x) / 3.0;
        im = (P.e[0].y + P.e[4].y + P.e[8].y) / 3.0;
    }
    const double tr = block_sum(re, sh);
    __syncthreads();
    const double ti = block_sum(im, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = tr;
        partial[2 * blockIdx.x + 1] = ti;
    }
}

__global__ void k_poly_final(const double *partial, int nb, int v3, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nb; b++) {
        re += partial[2 * b];
        im += partial[2 * b + 1];
    }
    out[0] = re / v3;
    out[1] = im / v3;
}

wd_status check_src(const wd_ctx *c, const int32_t src[4])
{
    if (!src) return set_error(WD_ERR_ARG, "NULL source");
    for (int mu = 0; mu < 4; mu++)
        if (src[mu] < 0 || src[mu] >= c->dims[mu])
            return set_error(WD_ERR_ARG, "source coordinate %d = %d outside 0..%d", mu, src[mu], c->dims[mu] - 1);
    return WD_OK;
}

wd_status read_back(wd_ctx *c, double *host, const double *dev, int n)
{
    void *h;
    WD_TRY(pinned_get(c, 1, sizeof(double) * n, &h));
    HIPCHK(hipMemcpyAsync(h, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(host, h, sizeof(double) * n);
    return WD_OK;
}

}  // namespace

}  // namespace wd

using namespace wd;

extern "C" wd_status wd_polyakov(wd_ctx *c, const double *U, double *out)
{
    if (!c || !U || !out) return set_error(WD_ERR_ARG, "NULL argument");
    WD_HIP(hipSetDevice(c->device));
    const int v3 = c->dims[0] * c->dims[1] * c->dims[2], Lt = c->dims[3];
    const int nb = (int)nblk(v3);
    void *vp;
    WD_TRY(ws_get(c, "ms_poly", sizeof(double) * (2 * nb + 2), &vp));
    double *partial = (double *)vp, *res = partial + 2 * nb;
    hipLaunchKernelGGL(k_poly_partial, dim3(nb), dim3(kB), 0, c->stream, U, v3, Lt, partial);
    hipLaunchKernelGGL(k_poly_final, dim3(1), dim3(64), 0, c->stream, partial, nb, v3, res);
    HIPCHK(hipGetLastError());
    return read_back(c, out, res, 2);
}

extern "C" wd_status wd_point_propagator(wd_ctx *c, double *psi, const int32_t src[4], double kappa,
                                         const wd_solver_params *pin, wd_solver_stats *st)
{
    if (!c || !psi) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    WD_TRY(check_src(c, src));
    if (!std::isfinite(kappa)) return set_error(WD_ERR_ARG, "kappa not finite");
    wd_solver_params p;
    wd_solver_defaults(&p);
    if (pin) p = *pin;
    if (!p.eo) return set_error(WD_ERR_ARG, "the propagator uses the even-odd solve (eo = 1)");
    WD_HIP(hipSetDevice(c->device));
    const hipStream_t s = c->stream;
    const long long Vh = c->Vh, V = 2 * Vh, col = Vh * 24;  // doubles per parity column
    const int x0 = src[0] + c->dims[0] * (src[1] + c->dims[1] * (src[2] + c->dims[2] * src[3]));
    const int par = (src[0] + src[1] + src[2] + src[3]) & 1, cb0 = x0 >> 1;
    void *vp;
    WD_TRY(ws_get(c, "ms_a", sizeof(double) * 12 * col, &vp));
    double *A = (double *)vp;  // bhat, then the even solution
    WD_TRY(ws_get(c, "ms_b", sizeof(double) * 12 * col, &vp));
    double *B = (double *)vp;  // Mhat^dag bhat
    WD_TRY(ws_get(c, "ms_t", sizeof(double) * 3 * col, &vp));
    double *T1 = (double *)vp, *T2 = T1 + col, *PO = T2 + col;

    // bhat_j = b_e + k D_eo b_o
    hipLaunchKernelGGL(k_fill, dim3(nblk(12 * col)), dim3(kB), 0, s, A, 0.0, 12 * col);
    HIPCHK(hipGetLastError());
    if (par == 0) {
        hipLaunchKernelGGL(k_add_point, dim3(1), dim3(64), 0, s, A, cb0, col);
    } else {
        for (int j = 0; j < 12; j++) {
            hipLaunchKernelGGL(k_fill, dim3(nblk(col)), dim3(kB), 0, s, PO, 0.0, col);
            hipLaunchKernelGGL(k_add_one, dim3(1), dim3(64), 0, s, PO, cb0, j);
            WD_TRY(wd_dslash(c, A + (size_t)j * col, PO, WD_EVEN, 0, WD_F64));
            hipLaunchKernelGGL(k_scale, dim3(nblk(col)), dim3(kB), 0, s, A + (size_t)j * col, kappa, col);
        }
    }
    HIPCHK(hipGetLastError());
    // B_j = Mhat^dag bhat_j = bhat_j - k^2 D_oe^dag D_eo^dag bhat_j
    for (int j = 0; j < 12; j++) {
        double *a = A + (size_t)j * col, *b = B + (size_t)j * col;
        WD_TRY(wd_dslash(c, T1, a, WD_ODD, 1, WD_F64));
        WD_TRY(wd_dslash(c, T2, T1, WD_EVEN, 1, WD_F64));
        HIPCHK(hipMemcpyAsync(b, a, sizeof(double) * col, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_axpy, dim3(nblk(col)), dim3(kB), 0, s, b, T2, -kappa * kappa, col);
    }
    HIPCHK(hipGetLastError());
    // psi_e: the batched solve of all 12 columns
    std::vector<double> kap(12, kappa);
    const wd_status sst = wd_cg_solve(c, A, B, 12, kap.data(), &p, st);
    if (sst != WD_OK && sst != WD_ERR_NOCONV && sst != WD_ERR_NAN) return sst;
    // psi_o = b_o + k D_oe psi_e, merged with psi_e into the full columns
    for (int j = 0; j < 12; j++) {
        const double *e = A + (size_t)j * col;
        WD_TRY(wd_dslash(c, T1, e, WD_ODD, 0, WD_F64));
        hipLaunchKernelGGL(k_scale, dim3(nblk(col)), dim3(kB), 0, s, T1, kappa, col);
        if (par == 1) hipLaunchKernelGGL(k_add_one, dim3(1), dim3(64), 0, s, T1, cb0, j);
        hipLaunchKernelGGL(k_merge, dim3(nblk(V)), dim3(kB), 0, s, e, T1, psi + (size_t)j * V * 24, c->g);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    if (sst != WD_OK) set_error(sst, "%s", sst == WD_ERR_NAN ? "non-finite residual" : "not converged");
    return sst;
}

extern "C" wd_status wd_pion_correlator(wd_ctx *c, double *corr, const double *psi, const int32_t src[4])
{
    if (!c || !corr || !psi) return set_error(WD_ERR_ARG, "NULL argument");
    WD_TRY(check_src(c, src));
    WD_HIP(hipSetDevice(c->device));
    const int v3 = c->dims[0] * c->dims[1] * c->dims[2], Lt = c->dims[3];
    const int nb = (int)nblk(v3);
    void *vp;
    WD_TRY(ws_get(c, "ms_corr", sizeof(double) * ((size_t)nb * Lt + Lt), &vp));
    double *partial = (double *)vp, *res = partial + (size_t)nb * Lt;
    hipLaunchKernelGGL(k_corr_partial, dim3(nb, Lt), dim3(kB), 0, c->stream, psi, (long long)2 * c->Vh, v3, nb,
                       partial);
    hipLaunchKernelGGL(k_corr_final, dim3((Lt + 63) / 64), dim3(64), 0, c->stream, partial, nb, Lt, src[3], res);
    HIPCHK(hipGetLastError());
    return read_back(c, corr, res, Lt);
}
