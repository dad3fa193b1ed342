// pack.hip -- conversion between the canonical complex128 layouts of the C-ABI
// and the internal structure-of-arrays layouts, and the device-side index
// tables used to check the kernels' neighbour arithmetic.
//
// The paper moves fields between host and GPU only at trajectory ends
// (Sec. 3); here the canonical fields are already device resident and these
// kernels run once per call, never inside an iteration.
#include "wd_internal.h"

namespace wd {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void lex_to_eo(const Geom &g, long long lex, int *P, int *cb)
{
    int x = (int)(lex % g.L[0]);
    long long r = lex / g.L[0];
    int y = (int)(r % g.L[1]);
    r /= g.L[1];
    int z = (int)(r % g.L[2]);
    int t = (int)(r / g.L[2]);
    *P = (x + y + z + t) & 1;
    *cb = (int)(lex >> 1);
}

// links: one thread per (lex, mu)
template <int LK>
__global__ void __launch_bounds__(kBlock) k_pack_gauge(const double *U, char *dst, Geom g)
{
    const long long V = 2LL * g.Vh;
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 4 * V) return;
    const long long lex = idx >> 2;
    const int mu = (int)(idx & 3);
    int P, cb;
    lex_to_eo(g, lex, &P, &cb);
    const double *u = U + idx * 18;
    const int blk = P * 4 + mu;
    const size_t cs = g.cs;
    if (LK == LK_F64_18 || LK == LK_F64_12) {
        const int nch = (LK == LK_F64_18) ? 9 : 6;
        double2 *d = reinterpret_cast<double2 *>(dst) + (size_t)blk * nch * cs;
        for (int k = 0; k < nch; k++) d[k * cs + cb] = make_double2(u[2 * k], u[2 * k + 1]);
    } else if (LK == LK_F32_12) {
        float4 *d = reinterpret_cast<float4 *>(dst) + (size_t)blk * 3 * cs;
        for (int k = 0; k < 3; k++)
            d[k * cs + cb] = make_float4((float)u[4 * k], (float)u[4 * k + 1], (float)u[4 * k + 2],
                                         (float)u[4 * k + 3]);
    } else if (LK == LK_F32_8) {
        // U' = s P C_k(U) (see LinkIO<LK_F32_8>): k takes the largest entry
        // of row 1 to U'_11; P swaps rows 2 and 3 (and s = -1) when |U'_31| <
        // |U'_21|; a block-diagonal U' keeps its lower block's first row
        double m[3];
        for (int j = 0; j < 3; j++) m[j] = u[2 * j] * u[2 * j] + u[2 * j + 1] * u[2 * j + 1];
        const int k = (m[1] > m[0] && m[1] >= m[2]) ? 1 : ((m[2] > m[0] && m[2] > m[1]) ? 2 : 0);
        double v[18];
        for (int row = 0; row < 3; row++)
            for (int j = 0; j < 3; j++) {
                v[6 * row + 2 * j] = u[6 * row + 2 * ((j + k) % 3)];
                v[6 * row + 2 * j + 1] = u[6 * row + 2 * ((j + k) % 3) + 1];
            }
        const double N = v[2] * v[2] + v[3] * v[3] + v[4] * v[4] + v[5] * v[5];
        const bool deg = !(N >= 1e-30);
        const bool swp = !deg && v[12] * v[12] + v[13] * v[13] < v[6] * v[6] + v[7] * v[7];
        if (swp)
            for (int e = 0; e < 6; e++) {
                const double r2 = v[6 + e];
                v[6 + e] = -v[12 + e];
                v[12 + e] = -r2;
                v[e] = -v[e];
            }
        const double inv2pi = 0.15915494309189535;
        // the phases in revolutions, k and (P, block) in their lowest mantissa bits
        const float pa = __uint_as_float((__float_as_uint((float)(atan2(v[1], v[0]) * inv2pi)) & ~3u) | (unsigned)k);
        const float pc = __uint_as_float((__float_as_uint(deg ? 0.0f : (float)(atan2(v[13], v[12]) * inv2pi)) & ~3u) |
                                         (swp ? 1u : 0u) | (deg ? 2u : 0u));
        float4 *d = reinterpret_cast<float4 *>(dst) + (size_t)blk * 2 * cs;
        if (deg)
            d[cb] = make_float4((float)v[8], (float)v[9], (float)v[10], (float)v[11]);
        else
            d[cb] = make_float4((float)v[2], (float)v[3], (float)v[4], (float)v[5]);
        d[cs + cb] = make_float4(deg ? 0.0f : (float)v[6], deg ? 0.0f : (float)v[7], pa, pc);
    } else if (LK == LK_F32_18) {
        float4 *d = reinterpret_cast<float4 *>(dst) + (size_t)blk * 4 * cs;
        for (int k = 0; k < 4; k++)
            d[k * cs + cb] = make_float4((float)u[4 * k], (float)u[4 * k + 1], (float)u[4 * k + 2],
                                         (float)u[4 * k + 3]);
        float2 *q = reinterpret_cast<float2 *>(reinterpret_cast<float4 *>(dst) + 32 * cs) + (size_t)blk * cs;
        q[cb] = make_float2((float)u[16], (float)u[17]);
    } else {
        half4_t *d = reinterpret_cast<half4_t *>(dst) + (size_t)blk * 3 * cs;
        for (int k = 0; k < 3; k++) {
            half4_t w;
            for (int j = 0; j < 4; j++) w[j] = (_Float16)u[4 * k + j];
            d[k * cs + cb] = w;
        }
    }
}

// spinors: one thread per site per RHS (grid.y = RHS)
template <int SP>
__global__ void __launch_bounds__(kBlock) k_pack_spinor(const double *src, char *base,
                                                         long long rs, long long ss, Geom g,
                                                         int mode)
{
    const long long n = mode ? 2LL * g.Vh : g.Vh;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int rid = blockIdx.y;
    int P = 0, cb = (int)s;
    if (mode) lex_to_eo(g, s, &P, &cb);
    double v[24];
    const double *p = src + ((long long)rid * n + s) * 24;
    for (int k = 0; k < 24; k++) v[k] = p[k];
    SpinorIO<SP>::store(base + rid * rs + P * ss, g.cs, cb, v);
}

template <int SP>
__global__ void __launch_bounds__(kBlock) k_unpack_spinor(const char *base, long long rs,
                                                           long long ss, double *dst, Geom g,
                                                           int mode)
{
    const long long n = mode ? 2LL * g.Vh : g.Vh;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int rid = blockIdx.y;
    int P = 0, cb = (int)s;
    if (mode) lex_to_eo(g, s, &P, &cb);
    double v[24];
    SpinorIO<SP>::load(base + rid * rs + P * ss, g.cs, cb, v);
    double *p = dst + ((long long)rid * n + s) * 24;
    for (int k = 0; k < 24; k++) p[k] = v[k];
}

template <int MU, int DIR>
__device__ __forceinline__ void nb_entry(const Geom &g, int i, int P, const int c[4], int32_t *row)
{
    const int j = neighbour<MU, DIR>(g, i, c);
    int cn[4];
    site_coords(g, j, 1 - P, cn);
    row[2 * MU + (DIR < 0)] = cn[0] + g.L[0] * (cn[1] + g.L[1] * (cn[2] + g.L[2] * cn[3]));
}

// What the stencil kernels compute: visit sites as (parity, cb) exactly as
// they do, derive coordinates and neighbours with the same device functions,
// and write the results in lex order.
__global__ void __launch_bounds__(kBlock) k_debug_tables(Geom g, int32_t *nb, int32_t *cbt,
                                                          uint8_t *par)
{
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= 2LL * g.Vh) return;
    const int P = (int)(s / g.Vh), i = (int)(s - (long long)P * g.Vh);
    int c[4];
    site_coords(g, i, P, c);
    const long long lex = c[0] + (long long)g.L[0] * (c[1] + (long long)g.L[1] * (c[2] + (long long)g.L[2] * c[3]));
    cbt[lex] = i;
    par[lex] = (uint8_t)P;
    int32_t row[8];
    nb_entry<0, +1>(g, i, P, c, row);
    nb_entry<0, -1>(g, i, P, c, row);
    nb_entry<1, +1>(g, i, P, c, row);
    nb_entry<1, -1>(g, i, P, c, row);
    nb_entry<2, +1>(g, i, P, c, row);
    nb_entry<2, -1>(g, i, P, c, row);
    nb_entry<3, +1>(g, i, P, c, row);
    nb_entry<3, -1>(g, i, P, c, row);
    for (int k = 0; k < 8; k++) nb[lex * 8 + k] = row[k];
}

}  // namespace

hipError_t pack_gauge(const double *U, char *dst, int lk, const Geom &g, hipStream_t s)
{
    const long long n = 8LL * g.Vh;  // 4 V links
    dim3 gr((unsigned)((n + kBlock - 1) / kBlock));
    switch (lk) {
    case LK_F64_18: hipLaunchKernelGGL(k_pack_gauge<LK_F64_18>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    case LK_F64_12: hipLaunchKernelGGL(k_pack_gauge<LK_F64_12>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    case LK_F32_12: hipLaunchKernelGGL(k_pack_gauge<LK_F32_12>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    case LK_F16_12: hipLaunchKernelGGL(k_pack_gauge<LK_F16_12>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    case LK_F32_18: hipLaunchKernelGGL(k_pack_gauge<LK_F32_18>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    case LK_F32_8: hipLaunchKernelGGL(k_pack_gauge<LK_F32_8>, gr, dim3(kBlock), 0, s, U, dst, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t pack_spinor(const double *src, const Field &dst, int nrhs, int mode, const Geom &g,
                       hipStream_t s)
{
    if (nrhs == 0) return hipSuccess;
    const long long n = mode ? 2LL * g.Vh : g.Vh;
    dim3 gr((unsigned)((n + kBlock - 1) / kBlock), nrhs);
    switch (dst.sp) {
    case SP_F64: hipLaunchKernelGGL(k_pack_spinor<SP_F64>, gr, dim3(kBlock), 0, s, src, dst.base, dst.rs, dst.ss, g, mode); break;
    case SP_F32: hipLaunchKernelGGL(k_pack_spinor<SP_F32>, gr, dim3(kBlock), 0, s, src, dst.base, dst.rs, dst.ss, g, mode); break;
    case SP_F16: hipLaunchKernelGGL(k_pack_spinor<SP_F16>, gr, dim3(kBlock), 0, s, src, dst.base, dst.rs, dst.ss, g, mode); break;
    case SP_I16: hipLaunchKernelGGL(k_pack_spinor<SP_I16>, gr, dim3(kBlock), 0, s, src, dst.base, dst.rs, dst.ss, g, mode); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t unpack_spinor(const Field &src, double *dst, int nrhs, int mode, const Geom &g,
                         hipStream_t s)
{
    if (nrhs == 0) return hipSuccess;
    const long long n = mode ? 2LL * g.Vh : g.Vh;
    dim3 gr((unsigned)((n + kBlock - 1) / kBlock), nrhs);
    switch (src.sp) {
    case SP_F64: hipLaunchKernelGGL(k_unpack_spinor<SP_F64>, gr, dim3(kBlock), 0, s, src.base, src.rs, src.ss, dst, g, mode); break;
    case SP_F32: hipLaunchKernelGGL(k_unpack_spinor<SP_F32>, gr, dim3(kBlock), 0, s, src.base, src.rs, src.ss, dst, g, mode); break;
    case SP_F16: hipLaunchKernelGGL(k_unpack_spinor<SP_F16>, gr, dim3(kBlock), 0, s, src.base, src.rs, src.ss, dst, g, mode); break;
    case SP_I16: hipLaunchKernelGGL(k_unpack_spinor<SP_I16>, gr, dim3(kBlock), 0, s, src.base, src.rs, src.ss, dst, g, mode); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t debug_tables(const Geom &g, int32_t *nb, int32_t *cb, uint8_t *par, hipStream_t s)
{
    const long long n = 2LL * g.Vh;
    hipLaunchKernelGGL(k_debug_tables, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, nb, cb, par);
    return hipGetLastError();
}

}  // namespace wd
