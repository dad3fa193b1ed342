// dslash_impl.h -- the even-odd Wilson hopping stencil (D_eo / D_oe and their
// adjoints) as one templated gfx950 kernel, with fused epilogues.
//
// Work mapping: RL consecutive lanes share one output site and each lane
// carries NR right-hand sides in registers, so one link load (and its 12-real
// reconstruction) serves NR RHS per lane, and the RL lanes that ask for the
// same link address are merged into one memory request.  A work-group covers
// blockDim/RL sites for RL*NR RHS.  For each of the 8 directions a lane loads
// the link once, then per RHS loads the neighbour spinor, projects it to a
// half spinor with (1 -+ gamma_mu), applies U or U^dag to the two colour
// vectors and accumulates the rebuilt 4-spinor.  FP64 fields use FP64
// arithmetic, FP32 / FP16 fields FP32 arithmetic (FP16 values are projected
// first and scaled by their site norm after).
//
// Epilogues:
//   EPI_PLAIN  out = D in
//   EPI_XPAY   out = x + coef[rid] * D in        (+ |out|^2 partial sums)
//   EPI_CGUPD  Ap  = x + coef[rid] * D in;  r -= alpha Ap  (+ |r|^2 partial
//              sums) -- the last sweep of Mhat^dag Mhat p fused with the CG
//              residual update (the solution is advanced from the search
//              directions of several iterations at once, by the p update).
// Partial sums cover 16 consecutive sites of one RHS and are formed with the
// same pairing tree for every (NR, RL, block) choice, so every launch shape
// gives bitwise-identical vectors and norms.
#pragma once

#include "wd_internal.h"

namespace wd {

// Neighbour spinor in compute precision.  For FP16 the per-site norm is
// returned separately (scale) so that it can be applied after projection.
template <int SP, typename real>
__device__ __forceinline__ real load_nb(const char *f, int cs, int j, real v[24])
{
    if constexpr (SP == SP_F16) {
        const half8_t *p = reinterpret_cast<const half8_t *>(f);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half8_t w = p[(size_t)k * cs + j];
#pragma unroll
            for (int q = 0; q < 8; q++) v[8 * k + q] = (real)(float)w[q];
        }
        return (real)reinterpret_cast<const float *>(f + (size_t)48 * cs)[j];
    } else if constexpr (SP == SP_I16) {
        const short8_t *p = reinterpret_cast<const short8_t *>(f);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            short8_t w = p[(size_t)k * cs + j];
#pragma unroll
            for (int q = 0; q < 8; q++) v[8 * k + q] = (real)(float)w[q];
        }
        return (real)SpinorIO<SP_I16>::step(reinterpret_cast<const float *>(f + (size_t)48 * cs)[j]);
    } else {
        SpinorIO<SP>::load(f, cs, j, v);
        return (real)1;
    }
}

// FP16 neighbour spinor as stored (24 halves), and its per-site norm; UNI:
// the field base is the same in every lane.
template <bool UNI>
__device__ __forceinline__ float load_nb_half(const char *f, int cs, int j, _Float16 v[24])
{
    const uint32_t off = UNI ? pin_v((uint32_t)j * 16u) : (uint32_t)j * 16u;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const half8_t w = ld_off<half8_t, UNI>(f + (size_t)k * cs * 16, off);
#pragma unroll
        for (int q = 0; q < 8; q++) v[8 * k + q] = w[q];
    }
    return ld_off<float, UNI>(f + (size_t)48 * cs, UNI ? pin_v((uint32_t)j * 4u) : (uint32_t)j * 4u);
}

// int16 neighbour spinor as stored (widened to int), and its quantisation
// step (norm / 32767).
template <bool UNI>
__device__ __forceinline__ float load_nb_i16(const char *f, int cs, int j, int v[24])
{
    const uint32_t off = UNI ? pin_v((uint32_t)j * 16u) : (uint32_t)j * 16u;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const short8_t w = ld_off<short8_t, UNI>(f + (size_t)k * cs * 16, off);
#pragma unroll
        for (int q = 0; q < 8; q++) v[8 * k + q] = w[q];
    }
    return SpinorIO<SP_I16>::step(ld_off<float, UNI>(f + (size_t)48 * cs, UNI ? pin_v((uint32_t)j * 4u) : (uint32_t)j * 4u));
}

// FP16 neighbour spinor as 12 (re, im) half2 pairs, and its per-site norm.
template <bool UNI>
__device__ __forceinline__ float load_nb_h2(const char *f, int cs, int j, h2_t v[12])
{
    const uint32_t off = UNI ? pin_v((uint32_t)j * 16u) : (uint32_t)j * 16u;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const half8_t w = ld_off<half8_t, UNI>(f + (size_t)k * cs * 16, off);
#pragma unroll
        for (int q = 0; q < 4; q++) v[4 * k + q] = h2_t{w[2 * q], w[2 * q + 1]};
    }
    return ld_off<float, UNI>(f + (size_t)48 * cs, UNI ? pin_v((uint32_t)j * 4u) : (uint32_t)j * 4u);
}

// Where a sweep reads the neighbour spinors.  GlobalNb: from the input field
// in global memory, for every direction (UNI: the field base is the same in
// every lane).  Each load returns the values as stored and the per-site scale
// of the format (1 without a norm); rid is the RHS id, r its index in the
// lane's group, j the neighbour's checkerboard index.
template <bool UNI>
struct GlobalNb {
    template <int MU, int DIR>
    __device__ __forceinline__ float half(const DslashArgs &a, int rid, int, int j, _Float16 v[24]) const
    {
        return load_nb_half<UNI>(a.in + rid * a.in_rs, a.g.cs, j, v);
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float h2(const DslashArgs &a, int rid, int, int j, h2_t v[12]) const
    {
        return load_nb_h2<UNI>(a.in + rid * a.in_rs, a.g.cs, j, v);
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float i16(const DslashArgs &a, int rid, int, int j, int v[24]) const
    {
        return load_nb_i16<UNI>(a.in + rid * a.in_rs, a.g.cs, j, v);
    }
    template <int MU, int DIR, int SP, typename real>
    __device__ __forceinline__ real gen(const DslashArgs &a, int rid, int, int j, real v[24]) const
    {
        return load_nb<SP>(a.in + rid * a.in_rs, a.g.cs, j, v);
    }
};

// LdsNb: the input planes (z, t-1), (z, t), (z, t+1) of the sites a work-group
// walks are staged in LDS (slot[0..2]; base[] their first checkerboard
// index), so the x, y and t neighbours come from LDS; the z neighbours from
// global memory.  Within a slot, RHS r occupies rstride bytes laid out like
// the global structure of arrays with chunk stride S (the sites of a plane):
// 16-byte chunk q of site jl at (q * S + jl) * 16, then the per-site norms.
typedef __attribute__((address_space(3))) char lds_char;

template <int SP>
struct LdsNb {
    const lds_char *slot[3];
    int base[3];
    int S;
    int rstride;

    template <int MU, int DIR>
    __device__ __forceinline__ const lds_char *at(int r, int j, int *jl) const
    {
        constexpr int k = (MU == 3) ? DIR + 1 : 1;
        *jl = j - base[k];
        return slot[k] + r * rstride;
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float half(const DslashArgs &a, int rid, int r, int j, _Float16 v[24]) const
    {
        if constexpr (MU == 2) {
            return GlobalNb<true>{}.template half<MU, DIR>(a, rid, r, j, v);
        } else {
            int jl;
            const lds_char *p = at<MU, DIR>(r, j, &jl);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const half8_t w = *(const __attribute__((address_space(3))) half8_t *)(p + (q * S + jl) * 16);
#pragma unroll
                for (int e = 0; e < 8; e++) v[8 * q + e] = w[e];
            }
            return *(const __attribute__((address_space(3))) float *)(p + 48 * S + jl * 4);
        }
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float h2(const DslashArgs &a, int rid, int r, int j, h2_t v[12]) const
    {
        if constexpr (MU == 2) {
            return GlobalNb<true>{}.template h2<MU, DIR>(a, rid, r, j, v);
        } else {
            int jl;
            const lds_char *p = at<MU, DIR>(r, j, &jl);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const half8_t w = *(const __attribute__((address_space(3))) half8_t *)(p + (q * S + jl) * 16);
#pragma unroll
                for (int e = 0; e < 4; e++) v[4 * q + e] = h2_t{w[2 * e], w[2 * e + 1]};
            }
            return *(const __attribute__((address_space(3))) float *)(p + 48 * S + jl * 4);
        }
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float i16(const DslashArgs &a, int rid, int r, int j, int v[24]) const
    {
        return GlobalNb<true>{}.template i16<MU, DIR>(a, rid, r, j, v);  // (no LDS variant for int16)
    }
    template <int MU, int DIR, int SP_, typename real>
    __device__ __forceinline__ real gen(const DslashArgs &a, int rid, int r, int j, real v[24]) const
    {
        if constexpr (MU == 2 || SP_ != SP_F32) {
            return GlobalNb<true>{}.template gen<MU, DIR, SP_>(a, rid, r, j, v);
        } else {
            int jl;
            const lds_char *p = at<MU, DIR>(r, j, &jl);
#pragma unroll
            for (int q = 0; q < 6; q++) {
                const flt4_t w = *(const __attribute__((address_space(3))) flt4_t *)(p + (q * S + jl) * 16);
                v[4 * q] = w.x;
                v[4 * q + 1] = w.y;
                v[4 * q + 2] = w.z;
                v[4 * q + 3] = w.w;
            }
            return (real)1;
        }
    }
};

// FP16 spinors with FP16 links: dot2 matvec on FP16 inputs, FP32 results.
template <int MU, int NR, bool DAG, class NB>
__device__ __forceinline__ void hop_dir_f16dot(const DslashArgs &a, const NB &nb, int i, const int c[4],
                                               const int rid[NR], float acc[NR][24])
{
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    const int cs = a.g.cs;
    h2_t A[9], B[9];
    {
        const int j = neighbour<MU, +1>(a.g, i, c);
        link_forms_f16<false>(a.links, cs, a.P * 4 + MU, i, A, B);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            h2_t v[12], h[6];
            float w[12];
            const float sc = nb.template h2<MU, +1>(a, rid[r], r, j, v);
            project_h2<MU, SF>(v, h);
            su3_mul_half_dot2(A, B, h, w);
            accumulate_scaled<MU, SF>(acc[r], w, sc);
        }
    }
    {
        const int j = neighbour<MU, -1>(a.g, i, c);
        link_forms_f16<true>(a.links, cs, (1 - a.P) * 4 + MU, j, A, B);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            h2_t v[12], h[6];
            float w[12];
            const float sc = nb.template h2<MU, -1>(a, rid[r], r, j, v);
            project_h2<MU, SB>(v, h);
            su3_mul_half_dot2(A, B, h, w);
            accumulate_scaled<MU, SB>(acc[r], w, sc);
        }
    }
}

// The two terms of direction MU for the NR RHS of a lane; nb supplies the
// neighbour spinors.
template <int MU, int SP, int LK, int NR, bool DAG, class NB, typename real>
__device__ __forceinline__ void hop_dir(const DslashArgs &a, const NB &nb, int i, const int c[4],
                                        const int rid[NR], real acc[NR][24])
{
    if constexpr (SP == SP_F16 && LK == LK_F16_12) {
        hop_dir_f16dot<MU, NR, DAG>(a, nb, i, c, rid, acc);
        return;
    }
    constexpr int SF = DAG ? +1 : -1;  // forward: (1 - g) for H, (1 + g) for H^dag
    constexpr int SB = -SF;            // backward: the opposite projector
    const int cs = a.g.cs;
    real u[18];
    {
        const int j = neighbour<MU, +1>(a.g, i, c);
        LinkIO<LK>::load(a.links, cs, a.P * 4 + MU, i, u);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            real h[12], w[12], sc;
            if constexpr (SP == SP_F16) {
                _Float16 v[24];
                sc = nb.template half<MU, +1>(a, rid[r], r, j, v);
                project_mix<MU, SF>(v, h);
            } else if constexpr (SP == SP_I16) {
                int v[24];
                sc = nb.template i16<MU, +1>(a, rid[r], r, j, v);
                project_int<MU, SF>(v, h);
            } else {
                real v[24];
                sc = nb.template gen<MU, +1, SP>(a, rid[r], r, j, v);
                project<MU, SF>(v, h);
            }
            su3_mul_half<false>(u, h, w);
            if constexpr (has_norm(SP))
                accumulate_scaled<MU, SF>(acc[r], w, sc);
            else
                accumulate<MU, SF>(acc[r], w);
        }
    }
    {
        const int j = neighbour<MU, -1>(a.g, i, c);
        LinkIO<LK>::load(a.links, cs, (1 - a.P) * 4 + MU, j, u);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            real h[12], w[12], sc;
            if constexpr (SP == SP_F16) {
                _Float16 v[24];
                sc = nb.template half<MU, -1>(a, rid[r], r, j, v);
                project_mix<MU, SB>(v, h);
            } else if constexpr (SP == SP_I16) {
                int v[24];
                sc = nb.template i16<MU, -1>(a, rid[r], r, j, v);
                project_int<MU, SB>(v, h);
            } else {
                real v[24];
                sc = nb.template gen<MU, -1, SP>(a, rid[r], r, j, v);
                project<MU, SB>(v, h);
            }
            su3_mul_half<true>(u, h, w);
            if constexpr (has_norm(SP))
                accumulate_scaled<MU, SB>(acc[r], w, sc);
            else
                accumulate<MU, SB>(acc[r], w);
        }
    }
}

// Sum over the 16 sites of a site group for lanes of equal RHS slot
// (lane = site * RL + slot): the same pairing tree for every RL.
template <int RL>
__device__ __forceinline__ double group16_sum(double v)
{
#pragma unroll
    for (int off = 8 * RL; off >= RL; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The epilogue of output site i (live: a site of this lattice) for the NR
// RHS of a lane (rv: the slot holds an active RHS): plain store, xpay with
// |out|^2, or the CG residual update with |r|^2; the norm partials of 16
// consecutive sites are summed with the same pairing tree for every shape.
template <int SP, int NR, int RL, int EPI, typename real>
__device__ __forceinline__ void dslash_epilogue(const DslashArgs &a, int i, bool live, const int (&rid)[NR],
                                                const bool (&rv)[NR], real (&acc)[NR][24])
{
    const int Vh = a.g.Vh, cs = a.g.cs;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        double nrm = 0.0;
        if (live && rv[r]) {
            if (EPI == EPI_PLAIN) {
                SpinorIO<SP>::template store<true>(a.out + rid[r] * a.out_rs, cs, i, acc[r]);
            } else if (EPI == EPI_XPAY) {
                const real cf = (real)a.coef[rid[r]];
                real xv[24];
                SpinorIO<SP>::template load<true>(a.x + rid[r] * a.x_rs, cs, i, xv);
#pragma unroll
                for (int k = 0; k < 24; k++) {
                    xv[k] = fmaT(cf, acc[r][k], xv[k]);
                    nrm = fmaT((double)xv[k], (double)xv[k], nrm);
                }
                SpinorIO<SP>::template store<true>(a.out + rid[r] * a.out_rs, cs, i, xv);
            } else {
                const real cf = (real)a.coef[rid[r]];
                const real al = (real)a.alpha[rid[r]];
                real ap[24], rv_[24];
                SpinorIO<SP>::template load<true>(a.x + rid[r] * a.x_rs, cs, i, ap);
                SpinorIO<SP>::template load<true>(a.r + rid[r] * a.r_rs, cs, i, rv_);
#pragma unroll
                for (int k = 0; k < 24; k++) {
                    ap[k] = fmaT(cf, acc[r][k], ap[k]);
                    rv_[k] = fmaT(-al, ap[k], rv_[k]);
                    nrm = fmaT((double)rv_[k], (double)rv_[k], nrm);
                }
                SpinorIO<SP>::template store<true>(a.r + rid[r] * a.r_rs, cs, i, rv_);
            }
        }
        if (EPI != EPI_PLAIN && a.partial != nullptr) {
            const double s = group16_sum<RL>(nrm);
            if ((i & 15) == 0 && i < Vh && rv[r] && ((int)threadIdx.x % (16 * RL)) < RL)
                a.partial[(size_t)rid[r] * a.pstride + a.pw_off + (i >> 4)] = s;
        }
    }
}

template <int SP, int LK, int NR, int RL, bool DAG, int EPI>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a)
{
    typedef typename SpinorIO<SP>::real real;
    static_assert(sizeof(typename LinkIO<LK>::real) == sizeof(real), "link/spinor precision pair");
    // the leading work-groups, if any, finalize the CG alpha of one active
    // RHS each (first wavefront; the order of every CG scalar's sum), the
    // others are the stencil's tiles; they are independent of each other
    if ((int)blockIdx.x < a.fin_blocks) {
        if (threadIdx.x < 64) {
            const int rid = a.active[blockIdx.x];
            const double s = fin_wave_sum(a.fin_partial + (size_t)rid * a.fin_pstride, a.fin_nw, (int)threadIdx.x);
            if (threadIdx.x == 0) fin_alpha_update(s, rid, a.fin_rr, a.fin_alpha, a.fin_out);
        }
        return;
    }
    // tile blocks: index and count without the finalize blocks (a block's
    // XCD is still its index mod 8, shifted alike for all of them)
    const int bid = (int)blockIdx.x - a.fin_blocks, nblk = (int)gridDim.x - a.fin_blocks;
    int tile, grp;
    if (a.remap == 7) {
        // z-slab per XCD as order 2, but RHS-group-major: the XCD sweeps its
        // whole slab for one RHS group before the next, so only NR*RL RHS of
        // spinor data are in flight (the links are re-read per group).
        const int x = bid & 7, j = bid >> 3;
        const int tx = (nblk / 8) / a.G;  // tiles per XCD
        grp = j / tx;
        const int sidx = j - grp * tx;
        const int q = sidx % a.tpp, zt = sidx / a.tpp;
        const int zl = zt % a.nzl, t = zt / a.nzl;
        tile = ((t * a.g.L[2]) + x * a.nzl + zl) * a.tpp + q;
    } else if (a.remap >= 5) {
        // XCD x owns t-planes [x*ntl, (x+1)*ntl) (ntl = Lt / 8, held in nzl)
        // and walks them t-fastest: a tile's t-neighbours are the tiles just
        // before and after it on the same XCD, its z-neighbours ntl tiles
        // away.  Order 5 takes (tile-in-plane, z, t), order 6 (z,
        // tile-in-plane, t), slowest to fastest.
        const int x = bid & 7, j = bid >> 3;
        const int sidx = j / a.G;
        grp = j - sidx * a.G;
        const int tl = sidx % a.nzl, rest = sidx / a.nzl;
        int z, q;
        if (a.remap == 5) {
            z = rest % a.g.L[2];
            q = rest / a.g.L[2];
        } else {
            q = rest % a.tpp;
            z = rest / a.tpp;
        }
        tile = ((x * a.nzl + tl) * a.g.L[2] + z) * a.tpp + q;
    } else if (a.remap >= 2) {
        // XCD x (= block id mod 8, the dispatch round-robin) owns z-planes
        // [x*nzl, (x+1)*nzl) for all t.  Each plane's tpp tiles form nys
        // stripes (consecutive tiles, i.e. ranges of y); the XCD sweeps one
        // stripe of its slab through all t before the next.  Its j-th block
        // takes RHS group j mod G of the (j / G)-th tile in (stripe, t, z,
        // tile-in-stripe) order, z fastest among planes, so the t and z
        // neighbours of a tile were read a few tiles earlier on the same XCD
        // (same L2), and a narrower stripe keeps that window smaller.
        const int x = bid & 7, j = bid >> 3;
        const int sidx = j / a.G;
        grp = j - sidx * a.G;
        const int tps = a.tpp / a.nys;
        const int qs = sidx % tps, rest = sidx / tps;
        const int zl = rest % a.nzl, ts = rest / a.nzl;
        const int t = ts % a.g.L[3], st = ts / a.g.L[3];
        tile = ((t * a.g.L[2]) + x * a.nzl + zl) * a.tpp + st * tps + qs;
    } else {
        const int L = a.remap ? xcd_remap(bid, nblk) : bid;
        tile = L / a.G;
        grp = L - tile * a.G;
    }
    const int spb = blockDim.x / RL;
    const int i = tile * spb + (int)threadIdx.x / RL;
    const int lr = (int)threadIdx.x % RL;
    const bool live = i < a.g.Vh;

    int rid[NR];
    bool rv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int slot = (grp * RL + lr) * NR + r;
        // a slot past the active count computes on RHS 0 (present in every
        // batch) without branches; its results are neither stored nor summed
        rv[r] = slot < a.nact;
        rid[r] = rv[r] ? a.active[slot] : 0;
        // with one lane per site the slot depends on the block only, so the
        // RHS id is the same in every lane: keep it (and the field bases
        // derived from it) in scalar registers
        if constexpr (RL == 1) rid[r] = __builtin_amdgcn_readfirstlane(rid[r]);
    }

    real acc[NR][24];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 24; k++) acc[r][k] = 0;

    if (live) {
        int c[4];
        site_coords(a.g, i, a.P, c);
        const GlobalNb<RL == 1> nb;
        hop_dir<0, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
        hop_dir<1, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
        hop_dir<2, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
        hop_dir<3, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
    }

    dslash_epilogue<SP, NR, RL, EPI>(a, i, live, rid, rv, acc);
}

// ---------------------------------------------------------------------------
// The LDS-staged variant: a work-group walks t along one z-plane column
// ---------------------------------------------------------------------------
// Work-group (z, t-chunk, RHS group) computes the output sites of the planes
// (z, t) for t in [t0, t0 + Tc), 256 threads over the S = Lx/2 * Ly sites of
// a plane, one lane per site and NR RHS per lane.  The input planes (z, t-1),
// (z, t), (z, t+1) of its RHS group are held in a ring of three LDS slots:
// the x and y neighbours of a site lie in plane (z, t), the t neighbours in
// (z, t+-1), so six of the eight neighbour spinors come from LDS and each
// input site of the column is read from HBM once per work-group (plus the
// two planes before and after the chunk); the z neighbours are read from
// global memory, where the work-groups of the adjacent z-planes (same XCD,
// same t and RHS group) read them too.  While a plane is computed, the next
// one is loaded into registers, and stored into the slot freed by the plane
// just finished.  The arithmetic, the epilogue and its norm partials are
// those of dslash_kernel, so the results are the same bits.
//
// XCD mapping: XCD x = block mod 8 takes the z-planes [x nzl, (x+1) nzl) (Lz
// divisible by 8); its j-th block is z-plane j mod nzl (fastest), then the
// RHS group, then the t chunk, so that the groups of one chunk, which read
// the same links, run on one XCD at the same time.

constexpr int kLdsThreads = 256;
constexpr int kLdsMaxPlane = 512;

// The chunk count of a spinor format's 16-byte chunks (the norm aside).
template <int SP>
__host__ __device__ constexpr int spinor_chunks() { return SP == SP_F32 ? 6 : 3; }

template <int SP>
__host__ __device__ constexpr int lds_site_bytes() { return SP == SP_F32 ? 96 : 52; }

template <int SP, int NR, int SPT>
struct PlaneRegs {
    u32x4_t ch[NR][SPT][spinor_chunks<SP>()];
    float nrm[NR][SPT];
};

// Global -> registers: plane (z, t) of the input field for the lane's sites
// tid + 256 k (k < SPT) and the NR RHS of the group.
template <int SP, int NR, int SPT>
__device__ __forceinline__ void plane_fetch(const DslashArgs &a, const int rid[NR], int pbase, int S,
                                            PlaneRegs<SP, NR, SPT> &R)
{
    const int cs = a.g.cs;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const char *f = a.in + rid[r] * a.in_rs;
#pragma unroll
        for (int k = 0; k < SPT; k++) {
            const int jl = (int)threadIdx.x + kLdsThreads * k;
            if (jl < S) {
                const int j = pbase + jl;
#pragma unroll
                for (int q = 0; q < spinor_chunks<SP>(); q++)
                    R.ch[r][k][q] = *reinterpret_cast<const u32x4_t *>(f + ((size_t)q * cs + j) * 16);
                if constexpr (has_norm(SP))
                    R.nrm[r][k] = reinterpret_cast<const float *>(f + (size_t)48 * cs)[j];
            }
        }
    }
}

// Registers -> LDS slot (layout of LdsNb).
template <int SP, int NR, int SPT>
__device__ __forceinline__ void plane_store(lds_char *slot, int S, const PlaneRegs<SP, NR, SPT> &R)
{
    const int rstride = S * lds_site_bytes<SP>();
#pragma unroll
    for (int r = 0; r < NR; r++) {
        lds_char *p = slot + r * rstride;
#pragma unroll
        for (int k = 0; k < SPT; k++) {
            const int jl = (int)threadIdx.x + kLdsThreads * k;
            if (jl < S) {
#pragma unroll
                for (int q = 0; q < spinor_chunks<SP>(); q++)
                    *(__attribute__((address_space(3))) u32x4_t *)(p + (q * S + jl) * 16) = R.ch[r][k][q];
                if constexpr (has_norm(SP))
                    *(__attribute__((address_space(3))) float *)(p + 48 * S + jl * 4) = R.nrm[r][k];
            }
        }
    }
}

template <int SP, int LK, int NR, bool DAG, int EPI>
__global__ void __launch_bounds__(kLdsThreads) dslash_lds_kernel(DslashArgs a)
{
    typedef typename SpinorIO<SP>::real real;
    static_assert(SP == SP_F16 || SP == SP_F32, "LDS staging of FP16 and FP32 spinors");
    constexpr int SPT = kLdsMaxPlane / kLdsThreads;  // sites per thread and plane, at most
    extern __shared__ __attribute__((aligned(16))) char lds_dyn[];
    if ((int)blockIdx.x < a.fin_blocks) {
        if (threadIdx.x < 64) {
            const int rid = a.active[blockIdx.x];
            const double s = fin_wave_sum(a.fin_partial + (size_t)rid * a.fin_pstride, a.fin_nw, (int)threadIdx.x);
            if (threadIdx.x == 0) fin_alpha_update(s, rid, a.fin_rr, a.fin_alpha, a.fin_out);
        }
        return;
    }
    const int bid = (int)blockIdx.x - a.fin_blocks;
    const int Lz = a.g.L[2], Lt = a.g.L[3];
    const int S = a.g.Lxh * a.g.L[1];
    const int Tc = a.tpp;  // t planes per work-group
    const int nzl = a.nzl;
    const int x = bid & 7, jb = bid >> 3;
    const int zl = jb % nzl, rest = jb / nzl;
    const int grp = rest % a.G, tc = rest / a.G;
    const int z = x * nzl + zl, t0 = tc * Tc;

    int rid[NR];
    bool rv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int slot = grp * NR + r;
        rv[r] = slot < a.nact;
        rid[r] = __builtin_amdgcn_readfirstlane(rv[r] ? a.active[slot] : 0);
    }
    auto pbase = [&](int t) { return S * (z + Lz * (((t % Lt) + Lt) % Lt)); };
    lds_char *lds = (lds_char *)lds_dyn;
    const int slot_bytes = NR * S * lds_site_bytes<SP>();
    // prologue: planes t0 - 1, t0, t0 + 1 in slots 0, 1, 2
    {
        PlaneRegs<SP, NR, SPT> R;
#pragma unroll 1
        for (int q = 0; q < 3; q++) {
            plane_fetch<SP, NR, SPT>(a, rid, pbase(t0 - 1 + q), S, R);
            plane_store<SP, NR, SPT>(lds + q * slot_bytes, S, R);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int tr = 0; tr < Tc; tr++) {
        const int t = t0 + tr;
        PlaneRegs<SP, NR, SPT> nxt;
        const bool more = tr + 1 < Tc;
        if (more) plane_fetch<SP, NR, SPT>(a, rid, pbase(t + 2), S, nxt);
        LdsNb<SP> nb;
        nb.S = S;
        nb.rstride = S * lds_site_bytes<SP>();
#pragma unroll
        for (int q = 0; q < 3; q++) {
            nb.slot[q] = lds + ((tr + q) % 3) * slot_bytes;
            nb.base[q] = pbase(t - 1 + q);
        }
#pragma unroll
        for (int k = 0; k < SPT; k++) {
            const int il = (int)threadIdx.x + kLdsThreads * k;
            if (k * kLdsThreads < S) {  // (whole waves: S is a multiple of 64)
                const bool live = il < S;
                // (an idle lane's index is past the lattice: it stores and sums nothing)
                const int i = live ? pbase(t) + il : a.g.Vh;
                real acc[NR][24];
#pragma unroll
                for (int r = 0; r < NR; r++)
#pragma unroll
                    for (int e = 0; e < 24; e++) acc[r][e] = 0;
                if (live) {
                    int c[4];
                    site_coords(a.g, i, a.P, c);
                    hop_dir<0, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
                    hop_dir<1, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
                    hop_dir<2, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
                    hop_dir<3, SP, LK, NR, DAG>(a, nb, i, c, rid, acc);
                }
                dslash_epilogue<SP, NR, 1, EPI>(a, i, live, rid, rv, acc);
            }
        }
        __syncthreads();  // every lane is done with the slot of plane t - 1
        if (more) plane_store<SP, NR, SPT>(lds + (tr % 3) * slot_bytes, S, nxt);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The t-walking variant: t neighbours held in registers
// ---------------------------------------------------------------------------
// Work-group (tile, z, RHS group, t chunk) computes one tile of B = blockDim
// consecutive sites of the planes (z, t), t in [t0, t0 + Tc): lane l owns
// the site column at checkerboard offset o = tile * B + l of each plane.  The
// t neighbours of output site (x, y, z, t) are the input sites (x, y, z,
// t +- 1), and since the halving of x does not depend on t their offset in
// their planes is o as well: the lane loads the input spinors of its column
// at t + 1 once, uses them for the forward t hop at t and keeps them in
// registers for the backward t hop at t + 2.  Each input spinor is read from
// memory once for the t hops of a work-group (plus the plane before and the
// plane after the chunk), so the t neighbours, a whole slab of the lattice
// away in memory, need not survive in L2 until the next t plane is swept.
// The x, y and z neighbours come from global memory, where the lanes and
// work-groups of the same and the adjacent planes have just loaded them.
// The arithmetic, its order and the epilogue are those of dslash_kernel, so
// the results are the same bits.
//
// XCD mapping: XCD x = block mod 8 takes the z-planes [x nzl, (x+1) nzl) (Lz
// divisible by 8); its j-th block is tile j mod tpp (fastest), then the z
// plane, then the RHS group, then the t chunk, so the work-groups of one t
// chunk that share links (RHS groups) and neighbours (tiles, z-planes) run
// on one XCD at the same time.

// The input spinors of a lane's column in one t plane, as stored (FP16 and
// the per-site norm), for the NR RHS of its group.
template <int NR>
struct ColF16 {
    half8_t ch[NR][3];
    float nrm[NR];
};

template <int NR>
__device__ __forceinline__ void col_load_f16(const DslashArgs &a, const int rid[NR], int j, ColF16<NR> &C)
{
    const int cs = a.g.cs;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const char *f = a.in + rid[r] * a.in_rs;
        const uint32_t off = pin_v((uint32_t)j * 16u);
#pragma unroll
        for (int k = 0; k < 3; k++) C.ch[r][k] = ld_off<half8_t, true>(f + (size_t)k * cs * 16, off);
        C.nrm[r] = ld_off<float, true>(f + (size_t)48 * cs, pin_v((uint32_t)j * 4u));
    }
}

// Neighbour source of the t-walking kernel: t neighbours from the column
// registers (bwd: plane t - 1, fwd: plane t + 1), the others from global
// memory.
template <int NR>
struct TwNb {
    const ColF16<NR> &bwd;
    const ColF16<NR> &fwd;

    template <int MU, int DIR>
    __device__ __forceinline__ float half(const DslashArgs &a, int rid, int r, int j, _Float16 v[24]) const
    {
        if constexpr (MU == 3) {
            const ColF16<NR> &C = DIR > 0 ? fwd : bwd;
#pragma unroll
            for (int k = 0; k < 3; k++)
#pragma unroll
                for (int e = 0; e < 8; e++) v[8 * k + e] = C.ch[r][k][e];
            return C.nrm[r];
        } else {
            return GlobalNb<true>{}.template half<MU, DIR>(a, rid, r, j, v);
        }
    }
    template <int MU, int DIR>
    __device__ __forceinline__ float h2(const DslashArgs &a, int rid, int r, int j, h2_t v[12]) const
    {
        if constexpr (MU == 3) {
            const ColF16<NR> &C = DIR > 0 ? fwd : bwd;
#pragma unroll
            for (int k = 0; k < 3; k++)
#pragma unroll
                for (int e = 0; e < 4; e++) v[4 * k + e] = h2_t{C.ch[r][k][2 * e], C.ch[r][k][2 * e + 1]};
            return C.nrm[r];
        } else {
            return GlobalNb<true>{}.template h2<MU, DIR>(a, rid, r, j, v);
        }
    }
};

template <int SP, int LK, int NR, bool DAG, int EPI>
__global__ void __launch_bounds__(256) dslash_tw_kernel(DslashArgs a)
{
    static_assert(SP == SP_F16, "t-walking stencil: FP16 spinors");
    if ((int)blockIdx.x < a.fin_blocks) {
        if (threadIdx.x < 64) {
            const int rid = a.active[blockIdx.x];
            const double s = fin_wave_sum(a.fin_partial + (size_t)rid * a.fin_pstride, a.fin_nw, (int)threadIdx.x);
            if (threadIdx.x == 0) fin_alpha_update(s, rid, a.fin_rr, a.fin_alpha, a.fin_out);
        }
        return;
    }
    const int bid = (int)blockIdx.x - a.fin_blocks;
    const int Lz = a.g.L[2], Lt = a.g.L[3];
    const int S = a.g.Lxh * a.g.L[1];
    const int Tc = a.tch;
    const int x = bid & 7, jb = bid >> 3;
    const int q = jb % a.tpp, r1 = jb / a.tpp;
    const int zl = r1 % a.nzl, r2 = r1 / a.nzl;
    const int grp = r2 % a.G, tc = r2 / a.G;
    const int z = x * a.nzl + zl, t0 = tc * Tc;
    const int o = q * (int)blockDim.x + (int)threadIdx.x;  // < S: whole tiles per plane

    int rid[NR];
    bool rv[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const int slot = grp * NR + r;
        rv[r] = slot < a.nact;
        rid[r] = __builtin_amdgcn_readfirstlane(rv[r] ? a.active[slot] : 0);
    }
    // first checkerboard index of plane (z, t), 0 <= t < Lt
    auto pbase = [&](int t) { return S * (z + Lz * t); };
    ColF16<NR> P0, P1, P2;  // the column at t - 1, t, t + 1
    col_load_f16<NR>(a, rid, pbase(t0 == 0 ? Lt - 1 : t0 - 1) + o, P0);
    col_load_f16<NR>(a, rid, pbase(t0) + o, P1);
#pragma unroll 1
    for (int tr = 0; tr < Tc; tr++) {
        // The field bases and strides pass through an empty asm each plane,
        // so that the scalar addresses derived from them (one per chunk
        // array, RHS and link direction) are formed where they are used and
        // not all hoisted out of the loop, where they would not fit the
        // scalar registers (the compiler would spill them to vector lanes).
        DslashArgs b = a;
        asm volatile("" : "+s"(b.in), "+s"(b.in_rs), "+s"(b.links), "+s"(b.g.cs), "+s"(b.out), "+s"(b.out_rs),
                     "+s"(b.x), "+s"(b.x_rs), "+s"(b.r), "+s"(b.r_rs));
        const int t = t0 + tr;
        // (the site indexes, too: otherwise every address derived from them
        // becomes an induction variable held in vector registers)
        int jn = pbase(t + 1 == Lt ? 0 : t + 1) + o, i = pbase(t) + o;
        asm volatile("" : "+v"(jn), "+v"(i));
        col_load_f16<NR>(b, rid, jn, P2);
        typedef float real;
        real acc[NR][24];
#pragma unroll
        for (int r = 0; r < NR; r++)
#pragma unroll
            for (int e = 0; e < 24; e++) acc[r][e] = 0;
        // (every site is live; the test keeps the hops in a region of their
        // own, as in dslash_kernel, which the compiler schedules with far
        // fewer registers than the same code without it)
        const bool live = i < b.g.Vh;
        if (live) {
            int c[4];
            site_coords(b.g, i, b.P, c);
            const GlobalNb<true> gnb;
            hop_dir<0, SP, LK, NR, DAG>(b, gnb, i, c, rid, acc);
            hop_dir<1, SP, LK, NR, DAG>(b, gnb, i, c, rid, acc);
            hop_dir<2, SP, LK, NR, DAG>(b, gnb, i, c, rid, acc);
            const TwNb<NR> tnb{P0, P2};
            hop_dir<3, SP, LK, NR, DAG>(b, tnb, i, c, rid, acc);
        }
        dslash_epilogue<SP, NR, 1, EPI>(b, i, live, rid, rv, acc);
        P0 = P1;
        P1 = P2;
    }
}

// Runtime -> template dispatch over the epilogue for one instance.
#define WD_DSL_EPI(SP_, LK_, NR_, RL_, DAG_)                                                \
    switch (epi) {                                                                                \
    case EPI_PLAIN:                                                                               \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, RL_, DAG_, EPI_PLAIN>), dim3(grid),  \
                           dim3(block), a.lds, s, a);                                                 \
        return hipGetLastError();                                                                 \
    case EPI_XPAY:                                                                                \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, RL_, DAG_, EPI_XPAY>), dim3(grid),   \
                           dim3(block), a.lds, s, a);                                                 \
        return hipGetLastError();                                                                 \
    case EPI_CGUPD:                                                                               \
        hipLaunchKernelGGL((dslash_kernel<SP_, LK_, NR_, RL_, DAG_, EPI_CGUPD>), dim3(grid),  \
                           dim3(block), a.lds, s, a);                                                 \
        return hipGetLastError();                                                                 \
    default:                                                                                      \
        return hipErrorInvalidValue;                                                              \
    }

#define WD_DSL_SHAPE(SP_, LK_, NR_, RL_, DAG_)                                                   \
    if (nr == NR_ && rl == RL_) {                                                                 \
        WD_DSL_EPI(SP_, LK_, NR_, RL_, DAG_)                                                      \
    }

// (the dynamic LDS limit of each LDS instance is raised to the device's
// maximum once)
#define WD_DSL_LDS_ONE(SP_, LK_, NR_, DAG_, EPI_)                                                   \
    {                                                                                             \
        static bool lim_ = false;                                                                 \
        if (!lim_) {                                                                              \
            int dev_ = 0, mx_ = 0;                                                                \
            hipError_t e_ = hipGetDevice(&dev_);                                                  \
            if (e_ == hipSuccess)                                                                 \
                e_ = hipDeviceGetAttribute(&mx_, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_); \
            if (e_ == hipSuccess)                                                                 \
                e_ = hipFuncSetAttribute(                                                         \
                    reinterpret_cast<const void *>(&dslash_lds_kernel<SP_, LK_, NR_, DAG_, EPI_>),  \
                    hipFuncAttributeMaxDynamicSharedMemorySize, mx_);                             \
            if (e_ != hipSuccess) return e_;                                                      \
            lim_ = true;                                                                          \
        }                                                                                         \
        hipLaunchKernelGGL((dslash_lds_kernel<SP_, LK_, NR_, DAG_, EPI_>), dim3(grid),             \
                           dim3(kLdsThreads), lds_bytes, s, a);                                   \
        return hipGetLastError();                                                                 \
    }

#define WD_DSL_LDS_EPI(SP_, LK_, NR_, DAG_)                                                        \
    switch (epi) {                                                                                \
    case EPI_PLAIN: WD_DSL_LDS_ONE(SP_, LK_, NR_, DAG_, EPI_PLAIN)                                 \
    case EPI_XPAY: WD_DSL_LDS_ONE(SP_, LK_, NR_, DAG_, EPI_XPAY)                                   \
    case EPI_CGUPD: WD_DSL_LDS_ONE(SP_, LK_, NR_, DAG_, EPI_CGUPD)                                 \
    default: return hipErrorInvalidValue;                                                         \
    }

#define WD_DSL_TW_EPI(SP_, LK_, NR_, DAG_)                                                         \
    switch (epi) {                                                                                \
    case EPI_PLAIN:                                                                               \
        hipLaunchKernelGGL((dslash_tw_kernel<SP_, LK_, NR_, DAG_, EPI_PLAIN>), dim3(grid), dim3(block), \
                           a.lds, s, a);                                                          \
        return hipGetLastError();                                                                 \
    case EPI_XPAY:                                                                                \
        hipLaunchKernelGGL((dslash_tw_kernel<SP_, LK_, NR_, DAG_, EPI_XPAY>), dim3(grid), dim3(block),  \
                           a.lds, s, a);                                                          \
        return hipGetLastError();                                                                 \
    case EPI_CGUPD:                                                                               \
        hipLaunchKernelGGL((dslash_tw_kernel<SP_, LK_, NR_, DAG_, EPI_CGUPD>), dim3(grid), dim3(block), \
                           a.lds, s, a);                                                          \
        return hipGetLastError();                                                                 \
    default:                                                                                      \
        return hipErrorInvalidValue;                                                              \
    }

#define WD_DSL_TW_SHAPE(SP_, LK_, NR_, DAG_)                                                       \
    if (nr == NR_) {                                                                              \
        WD_DSL_TW_EPI(SP_, LK_, NR_, DAG_)                                                        \
    }

#define WD_DSL_LDS_SHAPE(SP_, LK_, NR_, DAG_)                                                      \
    if (nr == NR_) {                                                                              \
        WD_DSL_LDS_EPI(SP_, LK_, NR_, DAG_)                                                       \
    }

}  // namespace wd
