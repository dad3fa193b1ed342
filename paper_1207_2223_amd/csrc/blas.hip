// blas.hip -- CG vector kernels over batches of spinor fields (the level-1
// BLAS work the paper delegates to CUBLAS, Sec. 3), fused where CG allows,
// with deterministic FP64 reductions: each group of 16 consecutive sites
// writes one partial sum in a fixed pairing order, and blas_finalize adds the
// partials of one RHS in a fixed order in a single work-group.
#include "wd_internal.h"

namespace wd {

namespace {

constexpr int kBlock = 256;
constexpr int kFinBlock = kFinLanes;

__device__ __forceinline__ double sum16(double v)
{
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct FArg {
    char *base;
    long long rs, ss;
    int cs;
};
inline FArg fa(const Field &f) { return FArg{f.base, f.rs, f.ss, f.cs}; }

__device__ __forceinline__ char *site_base(const FArg &f, int rid, int sub)
{
    return f.base + rid * f.rs + sub * f.ss;
}

template <int SP>
__global__ void __launch_bounds__(kBlock) k_norm(FArg a, int Vh, int nsub, const int *active,
                                                  double *partial, int pstride)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (s < nsub * Vh) {
        const int sub = s / Vh, i = s - sub * Vh;
        real x[24];
        SpinorIO<SP>::load(site_base(a, rid, sub), a.cs, i, x);
#pragma unroll
        for (int k = 0; k < 24; k++) v = fmaT((double)x[k], (double)x[k], v);
    }
    v = sum16(v);
    if ((threadIdx.x & 15) == 0 && s < nsub * Vh) partial[(size_t)rid * pstride + (s >> 4)] = v;
}

template <int SP>
__global__ void __launch_bounds__(kBlock) k_p_update(FArg p, FArg r, const double *beta, int Vh,
                                                      int nsub, const int *active)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    const real b = (real)beta[rid];
    real pv[24], rv[24];
    SpinorIO<SP>::load(site_base(p, rid, sub), p.cs, i, pv);
    SpinorIO<SP>::load(site_base(r, rid, sub), r.cs, i, rv);
#pragma unroll
    for (int k = 0; k < 24; k++) pv[k] = fmaT(b, pv[k], rv[k]);
    SpinorIO<SP>::store(site_base(p, rid, sub), p.cs, i, pv);
}

// The directions p[0..m-1] of the last m iterations (ring slots, RHS stride rs).
struct Ring {
    const char *base[kMaxRing];
    long long rs;
};

// pd = r + beta p[m-1]; with FLUSH first x += alpha_j p[j] for j = 0..m-1,
// in that order (the order and roundings of advancing x once per iteration).
template <int SP, int XP, bool FLUSH>
__global__ void __launch_bounds__(kBlock) k_p_update_ring(Ring p, int m, FArg pd, FArg r, const double *beta,
                                                           FArg x, const double *ahist, int ahs, int Vh,
                                                           const int *active)
{
    typedef typename SpinorIO<SP>::real real;
    typedef typename SpinorIO<XP>::real xreal;
    const int rid = active[blockIdx.y];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Vh) return;
    real pv[24];
    if constexpr (FLUSH) {
        xreal xv[24];
        SpinorIO<XP>::load(x.base + rid * x.rs, x.cs, i, xv);
#pragma unroll
        for (int j = 0; j < kMaxRing; j++) {
            if (j < m) {
                const real al = (real)ahist[(size_t)j * ahs + rid];
                SpinorIO<SP>::load(p.base[j] + rid * p.rs, pd.cs, i, pv);
#pragma unroll
                for (int k = 0; k < 24; k++) xv[k] = fmaT((xreal)al, (xreal)pv[k], xv[k]);
            }
        }
        SpinorIO<XP>::store(x.base + rid * x.rs, x.cs, i, xv);
    } else {
        SpinorIO<SP>::load(p.base[m - 1] + rid * p.rs, pd.cs, i, pv);
    }
    real rv[24];
    SpinorIO<SP>::load(r.base + rid * r.rs, r.cs, i, rv);
    const real b = (real)beta[rid];
#pragma unroll
    for (int k = 0; k < 24; k++) pv[k] = fmaT(b, pv[k], rv[k]);
    SpinorIO<SP>::store(pd.base + rid * pd.rs, pd.cs, i, pv);
}

template <int SP, int XP>
__global__ void __launch_bounds__(kBlock) k_cg_update(FArg x, FArg p, FArg r, FArg Ap,
                                                       const double *alpha, int Vh, int nsub,
                                                       const int *active, double *partial,
                                                       int pstride)
{
    typedef typename SpinorIO<SP>::real real;
    typedef typename SpinorIO<XP>::real xreal;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (s < nsub * Vh) {
        const int sub = s / Vh, i = s - sub * Vh;
        const real al = (real)alpha[rid];
        real pv[24], rv[24], av[24];
        xreal xv[24];
        SpinorIO<SP>::load(site_base(p, rid, sub), p.cs, i, pv);
        SpinorIO<SP>::load(site_base(r, rid, sub), r.cs, i, rv);
        SpinorIO<SP>::load(site_base(Ap, rid, sub), Ap.cs, i, av);
        SpinorIO<XP>::load(site_base(x, rid, sub), x.cs, i, xv);
#pragma unroll
        for (int k = 0; k < 24; k++) {
            xv[k] = fmaT((xreal)al, (xreal)pv[k], xv[k]);
            rv[k] = fmaT(-al, av[k], rv[k]);
            v = fmaT((double)rv[k], (double)rv[k], v);
        }
        SpinorIO<XP>::store(site_base(x, rid, sub), x.cs, i, xv);
        SpinorIO<SP>::store(site_base(r, rid, sub), r.cs, i, rv);
    }
    v = sum16(v);
    if ((threadIdx.x & 15) == 0 && s < nsub * Vh) partial[(size_t)rid * pstride + (s >> 4)] = v;
}

template <int SPD, int SPS>
__global__ void __launch_bounds__(kBlock) k_copy(FArg d, FArg src, int Vh, int nsub,
                                                  const int *active)
{
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    double v[24];
    SpinorIO<SPS>::load(site_base(src, rid, sub), src.cs, i, v);
    SpinorIO<SPD>::store(site_base(d, rid, sub), d.cs, i, v);
}

// xhi (FP64) += xs ; xs = 0
template <int XP>
__global__ void __launch_bounds__(kBlock) k_add_zero(FArg xhi, FArg xs, int Vh, int nsub,
                                                      const int *active)
{
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    double h[24], l[24];
    SpinorIO<SP_F64>::load(site_base(xhi, rid, sub), xhi.cs, i, h);
    SpinorIO<XP>::load(site_base(xs, rid, sub), xs.cs, i, l);
#pragma unroll
    for (int k = 0; k < 24; k++) {
        h[k] += l[k];
        l[k] = 0.0;
    }
    SpinorIO<SP_F64>::store(site_base(xhi, rid, sub), xhi.cs, i, h);
    SpinorIO<XP>::store(site_base(xs, rid, sub), xs.cs, i, l);
}

// r = b - Ap, all FP64, with |r|^2 partials
__global__ void __launch_bounds__(kBlock) k_resid(FArg r, FArg b, FArg Ap, int Vh, int nsub,
                                                   const int *active, double *partial,
                                                   int pstride)
{
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (s < nsub * Vh) {
        const int sub = s / Vh, i = s - sub * Vh;
        double bv[24], av[24];
        SpinorIO<SP_F64>::load(site_base(b, rid, sub), b.cs, i, bv);
        SpinorIO<SP_F64>::load(site_base(Ap, rid, sub), Ap.cs, i, av);
#pragma unroll
        for (int k = 0; k < 24; k++) {
            bv[k] -= av[k];
            v = fmaT(bv[k], bv[k], v);
        }
        SpinorIO<SP_F64>::store(site_base(r, rid, sub), r.cs, i, bv);
    }
    v = sum16(v);
    if ((threadIdx.x & 15) == 0 && s < nsub * Vh) partial[(size_t)rid * pstride + (s >> 4)] = v;
}

template <int SP>
__global__ void __launch_bounds__(kBlock) k_zero(FArg a, int Vh, int nsub, const int *active)
{
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    double z[24];
#pragma unroll
    for (int k = 0; k < 24; k++) z[k] = 0.0;
    SpinorIO<SP>::store(site_base(a, rid, sub), a.cs, i, z);
}

// <a, b> = sum conj(a) b, real and imaginary partials
template <int SP>
__global__ void __launch_bounds__(kBlock) k_cdot(FArg a, FArg b, int Vh, int nsub, const int *active,
                                                  double *pre, double *pim, int pstride)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    double vr = 0.0, vi = 0.0;
    if (s < nsub * Vh) {
        const int sub = s / Vh, i = s - sub * Vh;
        real x[24], y[24];
        SpinorIO<SP>::load(site_base(a, rid, sub), a.cs, i, x);
        SpinorIO<SP>::load(site_base(b, rid, sub), b.cs, i, y);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double ar = x[2 * k], ai = x[2 * k + 1], br = y[2 * k], bi = y[2 * k + 1];
            vr = fmaT(ar, br, vr);
            vr = fmaT(ai, bi, vr);
            vi = fmaT(ar, bi, vi);
            vi = fmaT(-ai, br, vi);
        }
    }
    vr = sum16(vr);
    vi = sum16(vi);
    if ((threadIdx.x & 15) == 0 && s < nsub * Vh) {
        pre[(size_t)rid * pstride + (s >> 4)] = vr;
        pim[(size_t)rid * pstride + (s >> 4)] = vi;
    }
}

// p -= c r with c = <r, p> / rr (complex), per RHS
template <int SP>
__global__ void __launch_bounds__(kBlock) k_orth(FArg p, FArg r, const double *dre, const double *dim,
                                                  const double *rr, int Vh, int nsub, const int *active)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    const double n = rr[rid];
    const real cr = (real)(n > 0.0 ? dre[rid] / n : 0.0), ci = (real)(n > 0.0 ? dim[rid] / n : 0.0);
    real pv[24], rv[24];
    SpinorIO<SP>::load(site_base(p, rid, sub), p.cs, i, pv);
    SpinorIO<SP>::load(site_base(r, rid, sub), r.cs, i, rv);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const real ar = rv[2 * k], ai = rv[2 * k + 1];
        pv[2 * k] = fmaT(-cr, ar, fmaT(ci, ai, pv[2 * k]));
        pv[2 * k + 1] = fmaT(-cr, ai, fmaT(-ci, ar, pv[2 * k + 1]));
    }
    SpinorIO<SP>::store(site_base(p, rid, sub), p.cs, i, pv);
}

// p += a r  (a a real constant)
template <int SP>
__global__ void __launch_bounds__(kBlock) k_axpy_const(FArg p, FArg r, double a, int Vh, int nsub,
                                                        const int *active)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    real pv[24], rv[24];
    SpinorIO<SP>::load(site_base(p, rid, sub), p.cs, i, pv);
    SpinorIO<SP>::load(site_base(r, rid, sub), r.cs, i, rv);
#pragma unroll
    for (int k = 0; k < 24; k++) pv[k] = fmaT((real)a, rv[k], pv[k]);
    SpinorIO<SP>::store(site_base(p, rid, sub), p.cs, i, pv);
}

// p = r + (num[rid] / den[rid]) p
template <int SP>
__global__ void __launch_bounds__(kBlock) k_xpay_ratio(FArg p, FArg r, const double *num, const double *den,
                                                        int Vh, int nsub, const int *active)
{
    typedef typename SpinorIO<SP>::real real;
    const int rid = active[blockIdx.y];
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= nsub * Vh) return;
    const int sub = s / Vh, i = s - sub * Vh;
    const double d = den[rid];
    const real b = (real)(d > 0.0 ? num[rid] / d : 0.0);
    real pv[24], rv[24];
    SpinorIO<SP>::load(site_base(p, rid, sub), p.cs, i, pv);
    SpinorIO<SP>::load(site_base(r, rid, sub), r.cs, i, rv);
#pragma unroll
    for (int k = 0; k < 24; k++) pv[k] = fmaT(b, pv[k], rv[k]);
    SpinorIO<SP>::store(site_base(p, rid, sub), p.cs, i, pv);
}

// One work-group per active RHS: fixed-order sum of its partials, then the
// CG scalar update selected by mode.
__global__ void __launch_bounds__(kFinBlock) k_finalize(const double *partial, int pstride, int nw,
                                                         const int *active, int mode, double *rr,
                                                         double *alpha, double *beta, double *out)
{
    __shared__ double sh[kFinBlock];
    const int rid = active[blockIdx.x];
    const double v = fin_lane_sum(partial + (size_t)rid * pstride, nw, threadIdx.x);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kFinBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = sh[0];
        if (mode == FIN_STORE) {
            out[rid] = s;
        } else if (mode == FIN_ALPHA) {
            // s = p.Ap = |M p|^2; out: the iteration's slot of the alpha history
            fin_alpha_update(s, rid, rr, alpha, out);
        } else if (mode == FIN_BETA) {
            beta[rid] = s / rr[rid];
            rr[rid] = s;
        } else {
            rr[rid] = s;
        }
    }
}

inline dim3 grid_of(int Vh, int nsub, int nact) { return dim3((nsub * Vh + kBlock - 1) / kBlock, nact); }

}  // namespace

#define SP_SWITCH(sp, F)                                                                          \
    switch (sp) {                                                                                 \
    case SP_F64: F(SP_F64); break;                                                                \
    case SP_F32: F(SP_F32); break;                                                                \
    case SP_F16: F(SP_F16); break;                                                                \
    case SP_I16: F(SP_I16); break;                                                                \
    default: return hipErrorInvalidValue;                                                         \
    }

hipError_t blas_norm(const Field &a, int Vh, const int *active, int nact, double *partial,
                     int pstride, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
#define F(SP) hipLaunchKernelGGL(k_norm<SP>, grid_of(Vh, a.nsub, nact), dim3(kBlock), 0, s, fa(a), Vh, a.nsub, active, partial, pstride)
    SP_SWITCH(a.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_p_update(const Field &p, const Field &r, const double *beta, int Vh,
                         const int *active, int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (p.sp != r.sp) return hipErrorInvalidValue;
#define F(SP) hipLaunchKernelGGL(k_p_update<SP>, grid_of(Vh, p.nsub, nact), dim3(kBlock), 0, s, fa(p), fa(r), beta, Vh, p.nsub, active)
    SP_SWITCH(p.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_p_update_ring(const Field *p, int m, const Field &pdst, const Field &r, const double *beta,
                              bool flush, const Field &x, const double *ahist, int ahs, int Vh,
                              const int *active, int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (m < 1 || m > kMaxRing || pdst.nsub != 1) return hipErrorInvalidValue;
    Ring R{};
    for (int j = 0; j < m; j++) R.base[j] = p[j].base;
    R.rs = p[0].rs;
    const dim3 grid = grid_of(Vh, 1, nact);
#define F(SP_, XP_)                                                                                       \
    if (flush)                                                                                            \
        hipLaunchKernelGGL((k_p_update_ring<SP_, XP_, true>), grid, dim3(kBlock), 0, s, R, m, fa(pdst), fa(r), \
                           beta, fa(x), ahist, ahs, Vh, active);                                          \
    else                                                                                                  \
        hipLaunchKernelGGL((k_p_update_ring<SP_, XP_, false>), grid, dim3(kBlock), 0, s, R, m, fa(pdst),     \
                           fa(r), beta, fa(x), ahist, ahs, Vh, active);
    if (pdst.sp == SP_F64 && (!flush || x.sp == SP_F64)) {
        F(SP_F64, SP_F64)
    } else if (pdst.sp != SP_F64 && (!flush || x.sp == SP_F32)) {
        switch (pdst.sp) {
        case SP_F32: F(SP_F32, SP_F32) break;
        case SP_F16: F(SP_F16, SP_F32) break;
        case SP_I16: F(SP_I16, SP_F32) break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef F
    return hipGetLastError();
}

hipError_t blas_cg_update(const Field &x, const Field &p, const Field &r, const Field &Ap,
                          const double *alpha, int Vh, const int *active, int nact,
                          double *partial, int pstride, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    dim3 gr = grid_of(Vh, p.nsub, nact);
    if (p.sp == SP_F64 && x.sp == SP_F64)
        hipLaunchKernelGGL((k_cg_update<SP_F64, SP_F64>), gr, dim3(kBlock), 0, s, fa(x), fa(p), fa(r), fa(Ap), alpha, Vh, p.nsub, active, partial, pstride);
    else if (p.sp == SP_F32 && x.sp == SP_F32)
        hipLaunchKernelGGL((k_cg_update<SP_F32, SP_F32>), gr, dim3(kBlock), 0, s, fa(x), fa(p), fa(r), fa(Ap), alpha, Vh, p.nsub, active, partial, pstride);
    else if (p.sp == SP_F16 && x.sp == SP_F32)
        hipLaunchKernelGGL((k_cg_update<SP_F16, SP_F32>), gr, dim3(kBlock), 0, s, fa(x), fa(p), fa(r), fa(Ap), alpha, Vh, p.nsub, active, partial, pstride);
    else if (p.sp == SP_I16 && x.sp == SP_F32)
        hipLaunchKernelGGL((k_cg_update<SP_I16, SP_F32>), gr, dim3(kBlock), 0, s, fa(x), fa(p), fa(r), fa(Ap), alpha, Vh, p.nsub, active, partial, pstride);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t blas_copy(const Field &dst, const Field &src, int Vh, const int *active, int nact,
                     hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    dim3 gr = grid_of(Vh, dst.nsub, nact);
#define C2(D, S)                                                                                  \
    if (dst.sp == D && src.sp == S) {                                                             \
        hipLaunchKernelGGL((k_copy<D, S>), gr, dim3(kBlock), 0, s, fa(dst), fa(src), Vh, dst.nsub, active); \
        return hipGetLastError();                                                                 \
    }
    C2(SP_F64, SP_F64) C2(SP_F64, SP_F32) C2(SP_F64, SP_F16)
    C2(SP_F32, SP_F64) C2(SP_F32, SP_F32) C2(SP_F32, SP_F16)
    C2(SP_F16, SP_F64) C2(SP_F16, SP_F32) C2(SP_F16, SP_F16)
    C2(SP_F64, SP_I16) C2(SP_F32, SP_I16) C2(SP_I16, SP_F64) C2(SP_I16, SP_F32) C2(SP_I16, SP_I16)
#undef C2
    return hipErrorInvalidValue;
}

hipError_t blas_add_zero(const Field &xhi, const Field &xs, int Vh, const int *active, int nact,
                         hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (xhi.sp != SP_F64) return hipErrorInvalidValue;
    dim3 gr = grid_of(Vh, xhi.nsub, nact);
    if (xs.sp == SP_F32)
        hipLaunchKernelGGL(k_add_zero<SP_F32>, gr, dim3(kBlock), 0, s, fa(xhi), fa(xs), Vh, xhi.nsub, active);
    else if (xs.sp == SP_F64)
        hipLaunchKernelGGL(k_add_zero<SP_F64>, gr, dim3(kBlock), 0, s, fa(xhi), fa(xs), Vh, xhi.nsub, active);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t blas_resid(const Field &r, const Field &b, const Field &Ap, int Vh, const int *active,
                      int nact, double *partial, int pstride, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid, grid_of(Vh, r.nsub, nact), dim3(kBlock), 0, s, fa(r), fa(b), fa(Ap), Vh, r.nsub, active, partial, pstride);
    return hipGetLastError();
}

hipError_t blas_zero(const Field &a, int Vh, const int *active, int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
#define F(SP) hipLaunchKernelGGL(k_zero<SP>, grid_of(Vh, a.nsub, nact), dim3(kBlock), 0, s, fa(a), Vh, a.nsub, active)
    SP_SWITCH(a.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_cdot(const Field &a, const Field &b, int Vh, const int *active, int nact,
                     double *pre, double *pim, int pstride, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (a.sp != b.sp) return hipErrorInvalidValue;
#define F(SP) hipLaunchKernelGGL(k_cdot<SP>, grid_of(Vh, a.nsub, nact), dim3(kBlock), 0, s, fa(a), fa(b), Vh, a.nsub, active, pre, pim, pstride)
    SP_SWITCH(a.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_orth(const Field &p, const Field &r, const double *dre, const double *dim,
                     const double *rr, int Vh, const int *active, int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (p.sp != r.sp) return hipErrorInvalidValue;
#define F(SP) hipLaunchKernelGGL(k_orth<SP>, grid_of(Vh, p.nsub, nact), dim3(kBlock), 0, s, fa(p), fa(r), dre, dim, rr, Vh, p.nsub, active)
    SP_SWITCH(p.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_axpy_const(const Field &p, const Field &r, double a, int Vh, const int *active,
                           int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (p.sp != r.sp) return hipErrorInvalidValue;
#define F(SP) hipLaunchKernelGGL(k_axpy_const<SP>, grid_of(Vh, p.nsub, nact), dim3(kBlock), 0, s, fa(p), fa(r), a, Vh, p.nsub, active)
    SP_SWITCH(p.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_xpay_ratio(const Field &p, const Field &r, const double *num, const double *den, int Vh,
                           const int *active, int nact, hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    if (p.sp != r.sp) return hipErrorInvalidValue;
#define F(SP) hipLaunchKernelGGL(k_xpay_ratio<SP>, grid_of(Vh, p.nsub, nact), dim3(kBlock), 0, s, fa(p), fa(r), num, den, Vh, p.nsub, active)
    SP_SWITCH(p.sp, F)
#undef F
    return hipGetLastError();
}

hipError_t blas_finalize(const double *partial, int pstride, int nw, const int *active, int nact,
                         int mode, double *rr, double *alpha, double *beta, double *out,
                         hipStream_t s)
{
    if (nact == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(nact), dim3(kFinBlock), 0, s, partial, pstride, nw, active, mode, rr, alpha, beta, out);
    return hipGetLastError();
}

}  // namespace wd
