// dslash_impl.h -- the even-odd Wilson hopping stencil (D_eo / D_oe and their
// adjoints) as one templated gfx950 kernel, with fused epilogues.
//
// One thread computes one output site for NR right-hand sides: for each of
// the 8 directions it loads the link once (reconstructing row 3 from 12
// reals if compressed), then for every RHS loads the neighbour spinor,
// projects it to a half spinor with (1 -+ gamma_mu), applies U or U^dag to
// the two colour vectors and accumulates the rebuilt 4-spinor.  Arithmetic is
// FP64 for FP64 fields and FP32 otherwise.
//
// Epilogues:
//   EPI_PLAIN  out = D in
//   EPI_XPAY   out = x + coef[rid] * D in        (+ |out|^2 partial sums)
//   EPI_CGUPD  Ap  = x + coef[rid] * D in;  xs += alpha p;  r -= alpha Ap
//              (+ |r|^2 partial sums) -- the last sweep of Mhat^dag Mhat p
//              fused with the CG vector updates.
// Partial sums are per 64-site wavefront (independent of block size and of
// NR), so every launch shape gives bitwise-identical results.
#pragma once

#include "wd_internal.h"

namespace wd {

template <int MU, int SP, int LK, int NR, bool DAG, typename real>
__device__ __forceinline__ void hop_dir(const DslashArgs &a, int i, const int c[4],
                                        const int rid[NR], const bool rv[NR], real acc[NR][24])
{
    constexpr int SF = DAG ? +1 : -1;  // forward: (1 - g) for H, (1 + g) for H^dag
    constexpr int SB = -SF;            // backward: the opposite projector
    const int Vh = a.g.Vh;
    real u[18];
    {
        const int j = neighbour<MU, +1>(a.g, i, c);
        LinkIO<LK>::load(a.links, Vh, a.P * 4 + MU, i, u);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!rv[r]) continue;
            real v[24], h[12], w[12];
            SpinorIO<SP>::load(a.in + rid[r] * a.in_rs, Vh, j, v);
            project<MU, SF>(v, h);
            su3_mul_half<false>(u, h, w);
            accumulate<MU, SF>(acc[r], w);
        }
    }
    {
        const int j = neighbour<MU, -1>(a.g, i, c);
        LinkIO<LK>::load(a.links, Vh, (1 - a.P) * 4 + MU, j, u);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            if (!rv[r]) continue;
            real v[24], h[12], w[12];
            SpinorIO<SP>::load(a.in + rid[r] * a.in_rs, Vh, j, v);
            project<MU, SB>(v, h);
            su3_mul_half<true>(u, h, w);
            accumulate<MU, SB>(acc[r], w);
        }
    }
}

template <int SP, int LK, int NR, bool DAG, int EPI, int XP>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a)
{
    typedef typename SpinorIO<SP>::real real;
    static_assert(sizeof(typename LinkIO<LK>::real) == sizeof(real), "link/spinor precision pair");
    const int L = a.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int tile = L / a.G, grp = L - tile * a.G;
    const int i = tile * blockDim.x + threadIdx.x;
    const int Vh = a.g.Vh;
    const bool live = i < Vh;

    int rid[NR];
    bool rv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int slot = grp * NR + r;
        rv[r] = slot < a.nact;
        rid[r] = rv[r] ? a.active[slot] : 0;
    }

    real acc[NR][24];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 24; k++) acc[r][k] = 0;

    if (live) {
        int c[4];
        site_coords(a.g, i, a.P, c);
        hop_dir<0, SP, LK, NR, DAG>(a, i, c, rid, rv, acc);
        hop_dir<1, SP, LK, NR, DAG>(a, i, c, rid, rv, acc);
        hop_dir<2, SP, LK, NR, DAG>(a, i, c, rid, rv, acc);
        hop_dir<3, SP, LK, NR, DAG>(a, i, c, rid, rv, acc);
    }

#pragma unroll
    for (int r = 0; r < NR; r++) {
        double nrm = 0.0;
        if (live && rv[r]) {
            if (EPI == EPI_PLAIN) {
                SpinorIO<SP>::store(a.out + rid[r] * a.out_rs, Vh, i, acc[r]);
            } else if (EPI == EPI_XPAY) {
                const real cf = (real)a.coef[rid[r]];
                real xv[24];
                SpinorIO<SP>::load(a.x + rid[r] * a.x_rs, Vh, i, xv);
#pragma unroll
                for (int k = 0; k < 24; k++) {
                    xv[k] += cf * acc[r][k];
                    nrm += (double)xv[k] * (double)xv[k];
                }
                SpinorIO<SP>::store(a.out + rid[r] * a.out_rs, Vh, i, xv);
            } else {
                const real cf = (real)a.coef[rid[r]];
                const real al = (real)a.alpha[rid[r]];
                real ap[24], pv[24], rv_[24];
                typename SpinorIO<XP>::real xv[24];
                SpinorIO<SP>::load(a.x + rid[r] * a.x_rs, Vh, i, ap);
                SpinorIO<SP>::load(a.p + rid[r] * a.p_rs, Vh, i, pv);
                SpinorIO<SP>::load(a.r + rid[r] * a.r_rs, Vh, i, rv_);
                SpinorIO<XP>::load(a.xs + rid[r] * a.xs_rs, Vh, i, xv);
#pragma unroll
                for (int k = 0; k < 24; k++) {
                    ap[k] += cf * acc[r][k];
                    xv[k] += (typename SpinorIO<XP>::real)(al * pv[k]);
                    rv_[k] -= al * ap[k];
                    nrm += (double)rv_[k] * (double)rv_[k];
                }
                SpinorIO<XP>::store(a.xs + rid[r] * a.xs_rs, Vh, i, xv);
                SpinorIO<SP>::store(a.r + rid[r] * a.r_rs, Vh, i, rv_);
            }
        }
        if (a.partial != nullptr && EPI != EPI_PLAIN) {
            const double s = wave_sum(nrm);
            if ((threadIdx.x & 63) == 0 && i < Vh && rv[r])
                a.partial[(size_t)rid[r] * a.pstride + a.pw_off + (i >> 6)] = s;
        }
    }
}

// Runtime -> template dispatch for one (SP, XP) pair over link format, NR,
// dagger and epilogue.
#define WD_DSL_EPI(SP_, LK_, NR_, DAG_, XP_)                                                     \
    switch (epi) {                                                                                \
    case EPI_PLAIN:                                                                               \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, DAG_, EPI_PLAIN, XP_>), dim3(grid),      \
                           dim3(block), 0, s, a);                                                 \
        return hipGetLastError();                                                                 \
    case EPI_XPAY:                                                                                \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, DAG_, EPI_XPAY, XP_>), dim3(grid),       \
                           dim3(block), 0, s, a);                                                 \
        return hipGetLastError();                                                                 \
    case EPI_CGUPD:                                                                               \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, DAG_, EPI_CGUPD, XP_>), dim3(grid),      \
                           dim3(block), 0, s, a);                                                 \
        return hipGetLastError();                                                                 \
    default:                                                                                      \
        return hipErrorInvalidValue;                                                              \
    }

#define WD_DSL_DAG(SP_, LK_, NR_, XP_)                                                           \
    if (dag) {                                                                                    \
        WD_DSL_EPI(SP_, LK_, NR_, true, XP_)                                                      \
    } else {                                                                                      \
        WD_DSL_EPI(SP_, LK_, NR_, false, XP_)                                                     \
    }

}  // namespace wd
