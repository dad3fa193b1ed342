// wd_device.h -- device-side building blocks of the gfx950 stencil kernels:
// lattice index arithmetic, per-precision spinor and link storage, the spin
// projections of (1 +- gamma_mu) and the SU(3) matrix-vector products.
//
// Internal storage (structure of arrays, one parity "subfield" at a time):
//   spinor F64: double2 [12][cs]          (complex component k = 3*spin + colour)
//   spinor F32: float4  [6][cs]           (reals 4k..4k+3 of the 24)
//   spinor F16: half8   [3][cs] + float [cs] norm  (reals 8k..8k+7, times norm)
//   links  L64_18: double2 [9][cs], L64_12: double2 [6][cs],
//          L32_12: float4 [3][cs],  L16_12: half4 [3][cs],
//          L32_18: float4 [4][cs] (+ float2 [cs] in a second region)
//          per (parity, mu) block, blocks ordered (parity*4 + mu).
// cs >= Vh is the padded chunk stride (in sites): Vh is often a power of two
// and unpadded chunk arrays would all start at the same offset modulo large
// powers of two, so the chunks of one site would compete for the same L2
// sets and channels.
// Consecutive threads take consecutive checkerboard sites, so every load
// and store of a wavefront is one contiguous 1 KiB (16 B per lane) segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wd {

enum { SP_F64 = 0, SP_F32 = 1, SP_F16 = 2, SP_I16 = 3 };

// Formats that store a per-site FP32 norm next to 16-bit values.
__host__ __device__ constexpr bool has_norm(int sp) { return sp == SP_F16 || sp == SP_I16; }
enum { LK_F64_18 = 0, LK_F64_12 = 1, LK_F32_12 = 2, LK_F16_12 = 3, LK_F32_18 = 4, LK_F32_8 = 5 };
// FP32 12-real, FP64 12-real and FP32 8-real data read with non-temporal
// loads (launch variants of the same packed links, not storage formats).
enum { LK_F32_12N = 6, LK_F64_12N = 7, LK_F32_8N = 8 };

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// All library code is compiled without floating-point contraction; every
// fused multiply-add is written out with fmaT so that the rounding sequence
// is fixed by the source and identical in every kernel instantiation.
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Two FP32 values to a packed pair of FP16 (round to nearest even), low half
// first.  An ALU instruction only (no memory access).
__device__ __forceinline__ uint32_t cvt_pk_f16(float lo, float hi)
{
    uint32_t r;
    asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(r) : "v"(lo), "v"(hi));
    return r;
}
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

// Load of a T at byte offset off (32 bits: one chunk array is below 4 GiB)
// from base.  With UNI (base the same in every lane) the base is pinned to
// scalar registers, so that the load takes the scalar-base form with a
// 32-bit vector offset; otherwise the compiler folds base + chunk stride
// into a 64-bit address computed per lane.  The offset must be formed in
// the same basic block as the load (see pin_v) for that form to be chosen.
// Opaque copy of a 32-bit value: keeps an offset computed at its use, where
// the compiler would otherwise hoist it as a 64-bit value.
__device__ __forceinline__ uint32_t pin_v(uint32_t v)
{
    asm("" : "+v"(v));
    return v;
}

template <typename T, bool UNI>
__device__ __forceinline__ T ld_off(const char *base, uint32_t off)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef const __attribute__((address_space(1))) T gT;
    gchar *g = (gchar *)base;
    if constexpr (UNI) asm("" : "+s"(g));
    return *(gT *)(g + off);
}

// The same with a non-temporal hint (the value is the same; the caches are
// asked not to keep the line).
template <typename T, bool UNI>
__device__ __forceinline__ T ld_off_nt(const char *base, uint32_t off)
{
    typedef const __attribute__((address_space(1))) char gchar;
    typedef __attribute__((address_space(1))) T gT;
    gchar *g = (gchar *)base;
    if constexpr (UNI) asm("" : "+s"(g));
    return __builtin_nontemporal_load((gT *)(g + off));
}

// Exact division by a runtime constant d for 0 <= n < 2^31 by a multiply and
// a shift (Granlund & Montgomery, PLDI 1994): with l = ceil(log2 d) and
// m = ceil(2^(31+l) / d), floor(n/d) = (n * m) >> (31 + l).
struct FastDiv {
    unsigned m;
    int s;
};

__host__ __device__ __forceinline__ int fdiv(int n, FastDiv d)
{
    return (int)(((unsigned long long)(unsigned)n * d.m) >> d.s);
}

// Chunk stride for Vh sites: rounded up to 64 sites, then offset by an odd
// multiple of 64 sites (592 = 37 * 16) so that consecutive chunk arrays, the
// per-site norms and the fields of a batch start at staggered offsets.
inline int padded_stride(int Vh) { return (Vh + 63) / 64 * 64 + 37 * 16; }

inline FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1LL << l) < d) l++;
    const unsigned long long num = 1ULL << (31 + l);
    FastDiv f;
    f.m = (unsigned)((num + (unsigned long long)d - 1) / (unsigned long long)d);
    f.s = 31 + l;
    return f;
}

struct Geom {
    int L[4];
    int Vh;
    int cs;           // chunk stride of the structure-of-arrays layouts (sites)
    int Lxh;          // Lx / 2
    int sy, sz, st;   // checkerboard strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
    FastDiv dxh, dy, dz;  // division by Lxh, Ly, Lz
};

// Coordinates of checkerboard site i of parity P.  Because Lx is even,
// cb = (x >> 1) + Lxh * (y + Ly*(z + Lz*t)) and x's low bit follows from
// the parity.
__device__ __forceinline__ void site_coords(const Geom &g, int i, int P, int c[4])
{
    int q = fdiv(i, g.dxh);
    int x0 = 2 * (i - q * g.Lxh);
    int zt = fdiv(q, g.dy);
    int y = q - zt * g.L[1];
    int t = fdiv(zt, g.dz);
    int z = zt - t * g.L[2];
    c[0] = x0 + ((P + y + z + t) & 1);
    c[1] = y;
    c[2] = z;
    c[3] = t;
}

// Checkerboard index of the neighbour x +- mu of site i with coordinates c
// (periodic wrap).  The neighbour has the other parity.
template <int MU, int DIR>
__device__ __forceinline__ int neighbour(const Geom &g, int i, const int c[4])
{
    int L = g.L[MU];
    int v = c[MU] + DIR;
    v = (v == L) ? 0 : ((v < 0) ? L - 1 : v);
    if (MU == 0) return i - (c[0] >> 1) + (v >> 1);
    const int s = (MU == 1) ? g.sy : ((MU == 2) ? g.sz : g.st);
    return i + (v - c[MU]) * s;
}

// ---------------------------------------------------------------------------
// Spinor storage
// ---------------------------------------------------------------------------
// Vector loads and stores with an optional non-temporal hint (NT): data a
// sweep touches once at its own site (epilogue operands and outputs) is
// marked so that the L2 keeps the neighbour spinors and links, which are
// read by up to eight sites.  The hint changes caching only, never values.
typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

template <bool NT, typename V>
__device__ __forceinline__ V ld_hint(const V *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, typename V>
__device__ __forceinline__ void st_hint(V *p, V v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int SP> struct SpinorIO;

template <> struct SpinorIO<SP_F64> {
    typedef double real;
    static constexpr size_t site_bytes = 192;
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void load(const char *f, int cs, int i, T v[24])
    {
        const dbl2_t *p = reinterpret_cast<const dbl2_t *>(f);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const dbl2_t w = ld_hint<NT>(p + (size_t)k * cs + i);
            v[2 * k] = (T)w.x;
            v[2 * k + 1] = (T)w.y;
        }
    }
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void store(char *f, int cs, int i, const T v[24])
    {
        dbl2_t *p = reinterpret_cast<dbl2_t *>(f);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            dbl2_t w;
            w.x = (double)v[2 * k];
            w.y = (double)v[2 * k + 1];
            st_hint<NT>(p + (size_t)k * cs + i, w);
        }
    }
};

template <> struct SpinorIO<SP_F32> {
    typedef float real;
    static constexpr size_t site_bytes = 96;
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void load(const char *f, int cs, int i, T v[24])
    {
        const flt4_t *p = reinterpret_cast<const flt4_t *>(f);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const flt4_t w = ld_hint<NT>(p + (size_t)k * cs + i);
            v[4 * k] = (T)w.x;
            v[4 * k + 1] = (T)w.y;
            v[4 * k + 2] = (T)w.z;
            v[4 * k + 3] = (T)w.w;
        }
    }
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void store(char *f, int cs, int i, const T v[24])
    {
        flt4_t *p = reinterpret_cast<flt4_t *>(f);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            flt4_t w;
            w.x = (float)v[4 * k];
            w.y = (float)v[4 * k + 1];
            w.z = (float)v[4 * k + 2];
            w.w = (float)v[4 * k + 3];
            st_hint<NT>(p + (size_t)k * cs + i, w);
        }
    }
};

// FP16 with a per-site FP32 norm: stored value = v / n rounded to nearest
// even, n = max |v| over the 24 reals of the site; a zero site stores n = 0.
template <> struct SpinorIO<SP_F16> {
    typedef float real;
    static constexpr size_t site_bytes = 52;
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void load(const char *f, int cs, int i, T v[24])
    {
        const half8_t *p = reinterpret_cast<const half8_t *>(f);
        const float n = ld_hint<NT>(reinterpret_cast<const float *>(f + (size_t)48 * cs) + i);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const half8_t w = ld_hint<NT>(p + (size_t)k * cs + i);
#pragma unroll
            for (int j = 0; j < 8; j++) v[8 * k + j] = (T)((float)w[j] * n);
        }
    }
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void store(char *f, int cs, int i, const T v[24])
    {
        // The scaled value is rounded to FP32 and then to FP16 (RNE) by an
        // explicit conversion: left to itself the backend may fuse some of
        // the multiplies into one-rounding mixed FMAs in some instantiations.
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < 24; j++) m = fmaxf(m, fabsf((float)v[j]));
        const float inv = (m > 0.f) ? 1.0f / m : 0.f;
        u32x4_t *p = reinterpret_cast<u32x4_t *>(f);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            u32x4_t w;
#pragma unroll
            for (int j = 0; j < 4; j++)
                w[j] = cvt_pk_f16((float)v[8 * k + 2 * j] * inv, (float)v[8 * k + 2 * j + 1] * inv);
            st_hint<NT>(p + (size_t)k * cs + i, w);
        }
        st_hint<NT>(reinterpret_cast<float *>(f + (size_t)48 * cs) + i, m);
    }
};

// int16 fixed point with a per-site FP32 norm n = max |v| over the 24 reals:
// stored q = rint(v * (32767 / n)) in [-32767, 32767], read back as
// q * (n / 32767); a zero site stores n = 0.  Same 52 bytes per site as FP16,
// uniform absolute precision n / 65534 instead of FP16's relative 2^-11.
typedef short short8_t __attribute__((ext_vector_type(8)));

template <> struct SpinorIO<SP_I16> {
    typedef float real;
    static constexpr size_t site_bytes = 52;
    __device__ static __forceinline__ float step(float n) { return n / 32767.0f; }
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void load(const char *f, int cs, int i, T v[24])
    {
        const short8_t *p = reinterpret_cast<const short8_t *>(f);
        const float sc = step(ld_hint<NT>(reinterpret_cast<const float *>(f + (size_t)48 * cs) + i));
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const short8_t w = ld_hint<NT>(p + (size_t)k * cs + i);
#pragma unroll
            for (int j = 0; j < 8; j++) v[8 * k + j] = (T)((float)w[j] * sc);
        }
    }
    template <bool NT = false, typename T>
    __device__ static __forceinline__ void store(char *f, int cs, int i, const T v[24])
    {
        float m = 0.f;
#pragma unroll
        for (int j = 0; j < 24; j++) m = fmaxf(m, fabsf((float)v[j]));
        const float inv = (m > 0.f) ? 32767.0f / m : 0.f;
        u32x4_t *p = reinterpret_cast<u32x4_t *>(f);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            u32x4_t w;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int q0 = min(32767, max(-32767, (int)rintf((float)v[8 * k + 2 * j] * inv)));
                const int q1 = min(32767, max(-32767, (int)rintf((float)v[8 * k + 2 * j + 1] * inv)));
                w[j] = ((unsigned)q0 & 0xffffu) | ((unsigned)q1 << 16);
            }
            st_hint<NT>(p + (size_t)k * cs + i, w);
        }
        st_hint<NT>(reinterpret_cast<float *>(f + (size_t)48 * cs) + i, m);
    }
};

__host__ __device__ constexpr size_t spinor_site_bytes(int sp)
{
    return sp == SP_F64 ? 192 : (sp == SP_F32 ? 96 : 52);
}

// ---------------------------------------------------------------------------
// Link storage.  u[18] holds U row-major: u[2*(3a+b)] = Re U_ab, +1 = Im.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void reconstruct_row3(T u[18])
{
    // row 3 = conj(row1 x row2), exact for SU(3)
#define RE(a, b) u[2 * (3 * (a) + (b))]
#define IM(a, b) u[2 * (3 * (a) + (b)) + 1]
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int k = (j + 1) % 3, l = (j + 2) % 3;
        // (row1 x row2)_j = u0k u1l - u0l u1k
        T re = RE(0, k) * RE(1, l);
        re = fmaT(-IM(0, k), IM(1, l), re);
        re = fmaT(-RE(0, l), RE(1, k), re);
        re = fmaT(IM(0, l), IM(1, k), re);
        T im = RE(0, k) * IM(1, l);
        im = fmaT(IM(0, k), RE(1, l), im);
        im = fmaT(-RE(0, l), IM(1, k), im);
        im = fmaT(-IM(0, l), RE(1, k), im);
        RE(2, j) = re;
        IM(2, j) = -im;
    }
#undef RE
#undef IM
}

template <int LK> struct LinkIO;

template <> struct LinkIO<LK_F64_18> {
    typedef double real;
    static constexpr int nchunk = 9;
    static constexpr size_t chunk_bytes = 16;
    __device__ static __forceinline__ void load(const char *U, int cs, int blk, int i, double u[18])
    {
        const double2 *p = reinterpret_cast<const double2 *>(U) + (size_t)blk * 9 * cs;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            double2 w = p[(size_t)k * cs + i];
            u[2 * k] = w.x;
            u[2 * k + 1] = w.y;
        }
    }
};

template <bool NT>
struct LinkIOF64x12 {
    typedef double real;
    static constexpr int nchunk = 6;
    static constexpr size_t chunk_bytes = 16;
    __device__ static __forceinline__ void load(const char *U, int cs, int blk, int i, double u[18])
    {
        const dbl2_t *p = reinterpret_cast<const dbl2_t *>(U) + (size_t)blk * 6 * cs;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const dbl2_t w = ld_hint<NT>(p + (size_t)k * cs + i);
            u[2 * k] = w.x;
            u[2 * k + 1] = w.y;
        }
        reconstruct_row3(u);
    }
};
template <> struct LinkIO<LK_F64_12> : LinkIOF64x12<false> {};
template <> struct LinkIO<LK_F64_12N> : LinkIOF64x12<true> {};

template <bool NT>
struct LinkIOF32x12 {
    typedef float real;
    static constexpr int nchunk = 3;
    static constexpr size_t chunk_bytes = 16;
    __device__ static __forceinline__ void load(const char *U, int cs, int blk, int i, float u[18])
    {
        const char *p = U + (size_t)blk * 3 * cs * 16;
        const uint32_t off = (uint32_t)i * 16u;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const flt4_t w = NT ? ld_off_nt<flt4_t, true>(p + (size_t)k * cs * 16, off)
                                : ld_off<flt4_t, true>(p + (size_t)k * cs * 16, off);
            u[4 * k] = w.x;
            u[4 * k + 1] = w.y;
            u[4 * k + 2] = w.z;
            u[4 * k + 3] = w.w;
        }
        reconstruct_row3(u);
    }
};
template <> struct LinkIO<LK_F32_12> : LinkIOF32x12<false> {};
// Each link is read once per sweep and RHS group: with one group (all RHS of
// a site in one lane) the links are not read again, and loading them
// non-temporally leaves the L2 to the neighbour spinors.
template <> struct LinkIO<LK_F32_12N> : LinkIOF32x12<true> {};

template <> struct LinkIO<LK_F16_12> {
    typedef float real;
    static constexpr int nchunk = 3;
    static constexpr size_t chunk_bytes = 8;
    __device__ static __forceinline__ void load(const char *U, int cs, int blk, int i, float u[18])
    {
        const half4_t *p = reinterpret_cast<const half4_t *>(U) + (size_t)blk * 3 * cs;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            half4_t w = p[(size_t)k * cs + i];
#pragma unroll
            for (int j = 0; j < 4; j++) u[4 * k + j] = (float)w[j];
        }
        reconstruct_row3(u);
    }
};

// FP32 with all 18 reals (no reconstruction): reals 0..15 as float4 [4][cs]
// per (parity, mu) block, then reals 16..17 as float2 [cs] per block in a
// second region after all eight float4 blocks.
template <> struct LinkIO<LK_F32_18> {
    typedef float real;
    __device__ static __forceinline__ void load(const char *U, int cs, int blk, int i, float u[18])
    {
        const float4 *p = reinterpret_cast<const float4 *>(U) + (size_t)blk * 4 * cs;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            float4 w = p[(size_t)k * cs + i];
            u[4 * k] = w.x;
            u[4 * k + 1] = w.y;
            u[4 * k + 2] = w.z;
            u[4 * k + 3] = w.w;
        }
        const float2 *q = reinterpret_cast<const float2 *>(reinterpret_cast<const float4 *>(U) + (size_t)32 * cs) +
                          (size_t)blk * cs;
        float2 w = q[i];
        u[16] = w.x;
        u[17] = w.y;
    }
};

// FP32 with 8 reals.  The link U is stored as U' = s P C_k(U): C_k shifts
// the columns cyclically (C_k(U)_ij = U_i,(j+k)%3, det unchanged), with k
// chosen so that U'_11 = U_1k is the largest entry of row 1 (|a1|^2 >= 1/3:
// |a1| = sqrt(1 - N) is then accurate in FP32); P swaps rows 2 and 3 and
// s = -1 when |U'_31| < |U'_21| (s P has det 1), so that |c1|^2 >= N / 2.
// U' is kept as a2, a3 (float4 chunk 0), b1 and the phases of a1 and c1 in
// revolutions (arg / 2 pi; chunk 1), with k in the two lowest mantissa bits of
// the first phase and P in the lowest bit of the second (a change of at most
// 3 ulp of a phase).  The rest follows from unitarity and det U' = 1: with
// N = |a2|^2 + |a3|^2,
//   |a1| = sqrt(1 - N),  |c1| = sqrt(N - |b1|^2)  (row 1, column 1 unit),
//   b2 = -(c1* a3* + a2 a1* b1) / N,   b3 = (a2* c1* - a3 a1* b1) / N,
//   c2 = (a3* b1* - a2 a1* c1) / N,   c3 = -(a2* b1* + a3 a1* c1) / N
// (the 2x2 systems of row orthogonality with c* = a x b and b* = c x a);
// every term keeps the relative precision of the stored values, so the
// division by a small N costs no accuracy.  N = 0 (below 1e-30: U'
// block-diagonal, e.g. U = 1) leaves the lower block W undetermined: such a
// link stores W's first row (p, q) in chunk 0, b1 = 0, and bit 1 of the
// second phase set; then W = [[p, q], [-a1* q*, a1* p*]] (det W = a1*,
// |a1| = 1).  Finally U = C_-k(s P U').
template <bool NT>
struct LinkIOF32x8 {
    typedef float real;
    __device__ static __forceinline__ void load(const char *U8, int cs, int blk, int i, float u[18])
    {
        const char *p = U8 + (size_t)blk * 2 * cs * 16;
        const uint32_t off = (uint32_t)i * 16u;
        const flt4_t w0 = NT ? ld_off_nt<flt4_t, true>(p, off) : ld_off<flt4_t, true>(p, off);
        const flt4_t w1 = NT ? ld_off_nt<flt4_t, true>(p + (size_t)cs * 16, off)
                            : ld_off<flt4_t, true>(p + (size_t)cs * 16, off);
        const float a2r = w0.x, a2i = w0.y, a3r = w0.z, a3i = w0.w, b1r = w1.x, b1i = w1.y;
        const int k = (int)(__float_as_uint(w1.z) & 3u);
        const unsigned cb = __float_as_uint(w1.w) & 3u;
        const bool swp = (cb & 1u) != 0, deg = (cb & 2u) != 0;
        const float N = fmaT(a2r, a2r, fmaT(a2i, a2i, fmaT(a3r, a3r, a3i * a3i)));
        const float ca = __builtin_amdgcn_cosf(w1.z), sa = __builtin_amdgcn_sinf(w1.z);
        const float a1m = deg ? 1.0f : __builtin_sqrtf(fmaxf(1.0f - N, 0.0f));
        const float c1m = __builtin_sqrtf(fmaxf(N - fmaT(b1r, b1r, b1i * b1i), 0.0f));
        const float a1r = a1m * ca, a1i = a1m * sa;
        const float c1r = c1m * __builtin_amdgcn_cosf(w1.w), c1i = c1m * __builtin_amdgcn_sinf(w1.w);
        const float iN = __builtin_amdgcn_rcpf(N);
        // t = a1* b1 and s = a1* c1
        const float tr = fmaT(a1r, b1r, a1i * b1i), ti = fmaT(a1r, b1i, -a1i * b1r);
        const float sr = fmaT(a1r, c1r, a1i * c1i), si = fmaT(a1r, c1i, -a1i * c1r);
        float v[18];
        v[0] = a1r; v[1] = a1i; v[2] = a2r; v[3] = a2i; v[4] = a3r; v[5] = a3i;
        v[6] = b1r; v[7] = b1i;
        // b2 = -(conj(c1 a3) + a2 t) / N
        v[8] = -(fmaT(c1r, a3r, -c1i * a3i) + fmaT(a2r, tr, -a2i * ti)) * iN;
        v[9] = -(-fmaT(c1r, a3i, c1i * a3r) + fmaT(a2r, ti, a2i * tr)) * iN;
        // b3 = (conj(a2 c1) - a3 t) / N
        v[10] = (fmaT(a2r, c1r, -a2i * c1i) - fmaT(a3r, tr, -a3i * ti)) * iN;
        v[11] = (-fmaT(a2r, c1i, a2i * c1r) - fmaT(a3r, ti, a3i * tr)) * iN;
        v[12] = c1r; v[13] = c1i;
        // c2 = (conj(a3 b1) - a2 s) / N
        v[14] = (fmaT(a3r, b1r, -a3i * b1i) - fmaT(a2r, sr, -a2i * si)) * iN;
        v[15] = (-fmaT(a3r, b1i, a3i * b1r) - fmaT(a2r, si, a2i * sr)) * iN;
        // c3 = -(conj(a2 b1) + a3 s) / N
        v[16] = -(fmaT(a2r, b1r, -a2i * b1i) + fmaT(a3r, sr, -a3i * si)) * iN;
        v[17] = -(-fmaT(a2r, b1i, a2i * b1r) + fmaT(a3r, si, a3i * sr)) * iN;
        // block-diagonal U': row 1 (a1, 0, 0), W = [[p, q], [-a1* q*, a1* p*]]
        // with (p, q) in the a2, a3 slots
        {
            const float d[18] = {a1r, a1i, 0.0f, 0.0f, 0.0f, 0.0f,
                                 0.0f, 0.0f, a2r, a2i, a3r, a3i,
                                 0.0f, 0.0f,
                                 -fmaT(a1r, a3r, -a1i * a3i), -fmaT(-a1r, a3i, -a1i * a3r),
                                 fmaT(a1r, a2r, -a1i * a2i), fmaT(-a1r, a2i, -a1i * a2r)};
#pragma unroll
            for (int e = 0; e < 18; e++) v[e] = deg ? d[e] : v[e];
        }
        // undo s P: rows 2 and 3 back, all signs back
        const float sg = swp ? -1.0f : 1.0f;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const float r2 = v[6 + e], r3 = v[12 + e];
            v[e] *= sg;
            v[6 + e] = sg * (swp ? r3 : r2);
            v[12 + e] = sg * (swp ? r2 : r3);
        }
        // undo C_k: U_i,m = U'_i,(m - k) mod 3
#pragma unroll
        for (int row = 0; row < 3; row++)
#pragma unroll
            for (int m = 0; m < 3; m++)
#pragma unroll
                for (int ri = 0; ri < 2; ri++) {
                    const float x0 = v[6 * row + 2 * m + ri], x1 = v[6 * row + 2 * ((m + 2) % 3) + ri],
                                x2 = v[6 * row + 2 * ((m + 1) % 3) + ri];
                    u[6 * row + 2 * m + ri] = k == 0 ? x0 : (k == 1 ? x1 : x2);
                }
    }
};
template <> struct LinkIO<LK_F32_8> : LinkIOF32x8<false> {};
template <> struct LinkIO<LK_F32_8N> : LinkIOF32x8<true> {};

__host__ __device__ constexpr size_t link_bytes(int lk)
{
    return lk == LK_F64_18 ? 144
                           : (lk == LK_F64_12 || lk == LK_F64_12N
                                  ? 96
                                  : (lk == LK_F32_12 || lk == LK_F32_12N
                                         ? 48
                                         : (lk == LK_F16_12 ? 24 : (lk == LK_F32_8 || lk == LK_F32_8N ? 32 : 72))));
}

// ---------------------------------------------------------------------------
// Spin projection.  (1 + S g_mu) psi has only two independent spin rows
// (h0, h1); rows 2 and 3 are fixed multiples of them.  Derived from the
// chiral-basis gamma matrices:
//   mu=x: h0 = p0 + S i p3, h1 = p1 + S i p2;  row2 = -S i h1, row3 = -S i h0
//   mu=y: h0 = p0 - S p3,   h1 = p1 + S p2;    row2 =  S h1,   row3 = -S h0
//   mu=z: h0 = p0 + S i p2, h1 = p1 - S i p3;  row2 = -S i h0, row3 =  S i h1
//   mu=t: h0 = p0 + S p2,   h1 = p1 + S p3;    row2 =  S h0,   row3 =  S h1
// v[24]: spin s colour c re/im at 6s + 2c (+1); h[12]: h0 at 0..5, h1 at 6..11.
// ---------------------------------------------------------------------------
template <int MU, int S, typename T>
__device__ __forceinline__ void project(const T v[24], T h[12])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const T p0r = v[2 * c], p0i = v[2 * c + 1];
        const T p1r = v[6 + 2 * c], p1i = v[6 + 2 * c + 1];
        const T p2r = v[12 + 2 * c], p2i = v[12 + 2 * c + 1];
        const T p3r = v[18 + 2 * c], p3i = v[18 + 2 * c + 1];
        if (MU == 0) {  // + S i p3 ; + S i p2      (i*(a+ib) = -b + ia)
            h[2 * c] = p0r - S * p3i;
            h[2 * c + 1] = p0i + S * p3r;
            h[6 + 2 * c] = p1r - S * p2i;
            h[6 + 2 * c + 1] = p1i + S * p2r;
        } else if (MU == 1) {
            h[2 * c] = p0r - S * p3r;
            h[2 * c + 1] = p0i - S * p3i;
            h[6 + 2 * c] = p1r + S * p2r;
            h[6 + 2 * c + 1] = p1i + S * p2i;
        } else if (MU == 2) {  // + S i p2 ; - S i p3
            h[2 * c] = p0r - S * p2i;
            h[2 * c + 1] = p0i + S * p2r;
            h[6 + 2 * c] = p1r + S * p3i;
            h[6 + 2 * c + 1] = p1i - S * p3r;
        } else {
            h[2 * c] = p0r + S * p2r;
            h[2 * c + 1] = p0i + S * p2i;
            h[6 + 2 * c] = p1r + S * p3r;
            h[6 + 2 * c + 1] = p1i + S * p3i;
        }
    }
}

// project() on FP16 inputs with FP32 results.  Each term is one
// mixed-precision fused multiply-add, b * (+-1) + a, on the FP16 values:
// the conversions are exact and the sum is rounded once, so the result is
// the value of converting first and adding in FP32, in half the
// instructions.
template <int MU, int S>
__device__ __forceinline__ void project_mix(const _Float16 v[24], float h[12])
{
    // +-1 from a register the compiler cannot see into, so that the
    // multiply-add is not simplified into an FP32 add of converted values
    float one;
    asm("s_mov_b32 %0, 1.0" : "=s"(one));
    auto pm = [one](_Float16 a, _Float16 b, float sgn) { return __builtin_fmaf((float)b, sgn * one, (float)a); };
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const _Float16 p0r = v[2 * c], p0i = v[2 * c + 1];
        const _Float16 p1r = v[6 + 2 * c], p1i = v[6 + 2 * c + 1];
        const _Float16 p2r = v[12 + 2 * c], p2i = v[12 + 2 * c + 1];
        const _Float16 p3r = v[18 + 2 * c], p3i = v[18 + 2 * c + 1];
        if (MU == 0) {
            h[2 * c] = pm(p0r, p3i, -S);
            h[2 * c + 1] = pm(p0i, p3r, S);
            h[6 + 2 * c] = pm(p1r, p2i, -S);
            h[6 + 2 * c + 1] = pm(p1i, p2r, S);
        } else if (MU == 1) {
            h[2 * c] = pm(p0r, p3r, -S);
            h[2 * c + 1] = pm(p0i, p3i, -S);
            h[6 + 2 * c] = pm(p1r, p2r, S);
            h[6 + 2 * c + 1] = pm(p1i, p2i, S);
        } else if (MU == 2) {
            h[2 * c] = pm(p0r, p2i, -S);
            h[2 * c + 1] = pm(p0i, p2r, S);
            h[6 + 2 * c] = pm(p1r, p3i, S);
            h[6 + 2 * c + 1] = pm(p1i, p3r, -S);
        } else {
            h[2 * c] = pm(p0r, p2r, S);
            h[2 * c + 1] = pm(p0i, p2i, S);
            h[6 + 2 * c] = pm(p1r, p3r, S);
            h[6 + 2 * c + 1] = pm(p1i, p3i, S);
        }
    }
}

// project() on int16 inputs: each component is an integer sum or difference
// converted once (|a +- b| < 2^16, so both steps are exact and the value is
// that of converting first and adding in FP32), one add and one convert
// instead of two converts and an add.
template <int MU, int S>
__device__ __forceinline__ void project_int(const int v[24], float h[12])
{
    auto pm = [](int a, int b, int sgn) { return (float)(sgn > 0 ? a + b : a - b); };
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int p0r = v[2 * c], p0i = v[2 * c + 1];
        const int p1r = v[6 + 2 * c], p1i = v[6 + 2 * c + 1];
        const int p2r = v[12 + 2 * c], p2i = v[12 + 2 * c + 1];
        const int p3r = v[18 + 2 * c], p3i = v[18 + 2 * c + 1];
        if (MU == 0) {
            h[2 * c] = pm(p0r, p3i, -S);
            h[2 * c + 1] = pm(p0i, p3r, S);
            h[6 + 2 * c] = pm(p1r, p2i, -S);
            h[6 + 2 * c + 1] = pm(p1i, p2r, S);
        } else if (MU == 1) {
            h[2 * c] = pm(p0r, p3r, -S);
            h[2 * c + 1] = pm(p0i, p3i, -S);
            h[6 + 2 * c] = pm(p1r, p2r, S);
            h[6 + 2 * c + 1] = pm(p1i, p2i, S);
        } else if (MU == 2) {
            h[2 * c] = pm(p0r, p2i, -S);
            h[2 * c + 1] = pm(p0i, p2r, S);
            h[6 + 2 * c] = pm(p1r, p3i, S);
            h[6 + 2 * c + 1] = pm(p1i, p3r, -S);
        } else {
            h[2 * c] = pm(p0r, p2r, S);
            h[2 * c + 1] = pm(p0i, p2i, S);
            h[6 + 2 * c] = pm(p1r, p3r, S);
            h[6 + 2 * c + 1] = pm(p1i, p3i, S);
        }
    }
}

// acc += full 4-spinor rebuilt from the colour-rotated half spinor w.
template <int MU, int S, typename T>
__device__ __forceinline__ void accumulate(T acc[24], const T w[12])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const T a0r = w[2 * c], a0i = w[2 * c + 1];
        const T a1r = w[6 + 2 * c], a1i = w[6 + 2 * c + 1];
        acc[2 * c] += a0r;
        acc[2 * c + 1] += a0i;
        acc[6 + 2 * c] += a1r;
        acc[6 + 2 * c + 1] += a1i;
        if (MU == 0) {  // row2 = -S i h1, row3 = -S i h0    (-S i (a+ib) = S b - S i a)
            acc[12 + 2 * c] += S * a1i;
            acc[12 + 2 * c + 1] -= S * a1r;
            acc[18 + 2 * c] += S * a0i;
            acc[18 + 2 * c + 1] -= S * a0r;
        } else if (MU == 1) {  // row2 = S h1, row3 = -S h0
            acc[12 + 2 * c] += S * a1r;
            acc[12 + 2 * c + 1] += S * a1i;
            acc[18 + 2 * c] -= S * a0r;
            acc[18 + 2 * c + 1] -= S * a0i;
        } else if (MU == 2) {  // row2 = -S i h0, row3 = S i h1
            acc[12 + 2 * c] += S * a0i;
            acc[12 + 2 * c + 1] -= S * a0r;
            acc[18 + 2 * c] -= S * a1i;
            acc[18 + 2 * c + 1] += S * a1r;
        } else {  // row2 = S h0, row3 = S h1
            acc[12 + 2 * c] += S * a0r;
            acc[12 + 2 * c + 1] += S * a0i;
            acc[18 + 2 * c] += S * a1r;
            acc[18 + 2 * c + 1] += S * a1i;
        }
    }
}

// acc += sc * (full 4-spinor rebuilt from w): the FP16 per-site norm folded
// into the accumulation, one fused multiply-add per term.
template <int MU, int S, typename T>
__device__ __forceinline__ void accumulate_scaled(T acc[24], const T w[12], const T sc)
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const T a0r = w[2 * c], a0i = w[2 * c + 1];
        const T a1r = w[6 + 2 * c], a1i = w[6 + 2 * c + 1];
        acc[2 * c] = fmaT(sc, a0r, acc[2 * c]);
        acc[2 * c + 1] = fmaT(sc, a0i, acc[2 * c + 1]);
        acc[6 + 2 * c] = fmaT(sc, a1r, acc[6 + 2 * c]);
        acc[6 + 2 * c + 1] = fmaT(sc, a1i, acc[6 + 2 * c + 1]);
        if (MU == 0) {  // row2 = -S i h1, row3 = -S i h0    (-S i (a+ib) = S b - S i a)
            acc[12 + 2 * c] = fmaT(S * sc, a1i, acc[12 + 2 * c]);
            acc[12 + 2 * c + 1] = fmaT(-S * sc, a1r, acc[12 + 2 * c + 1]);
            acc[18 + 2 * c] = fmaT(S * sc, a0i, acc[18 + 2 * c]);
            acc[18 + 2 * c + 1] = fmaT(-S * sc, a0r, acc[18 + 2 * c + 1]);
        } else if (MU == 1) {  // row2 = S h1, row3 = -S h0
            acc[12 + 2 * c] = fmaT(S * sc, a1r, acc[12 + 2 * c]);
            acc[12 + 2 * c + 1] = fmaT(S * sc, a1i, acc[12 + 2 * c + 1]);
            acc[18 + 2 * c] = fmaT(-S * sc, a0r, acc[18 + 2 * c]);
            acc[18 + 2 * c + 1] = fmaT(-S * sc, a0i, acc[18 + 2 * c + 1]);
        } else if (MU == 2) {  // row2 = -S i h0, row3 = S i h1
            acc[12 + 2 * c] = fmaT(S * sc, a0i, acc[12 + 2 * c]);
            acc[12 + 2 * c + 1] = fmaT(-S * sc, a0r, acc[12 + 2 * c + 1]);
            acc[18 + 2 * c] = fmaT(-S * sc, a1i, acc[18 + 2 * c]);
            acc[18 + 2 * c + 1] = fmaT(S * sc, a1r, acc[18 + 2 * c + 1]);
        } else {  // row2 = S h0, row3 = S h1
            acc[12 + 2 * c] = fmaT(S * sc, a0r, acc[12 + 2 * c]);
            acc[12 + 2 * c + 1] = fmaT(S * sc, a0i, acc[12 + 2 * c + 1]);
            acc[18 + 2 * c] = fmaT(S * sc, a1r, acc[18 + 2 * c]);
            acc[18 + 2 * c + 1] = fmaT(S * sc, a1i, acc[18 + 2 * c + 1]);
        }
    }
}

// w = U h for both half-spinor rows (h, w: 12 reals), or U^dag h.
template <bool ADJ, typename T>
__device__ __forceinline__ void su3_mul_half(const T u[18], const T h[12], T w[12])
{
#pragma unroll
    for (int r = 0; r < 2; r++) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            T re = 0, im = 0;
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const int idx = ADJ ? 2 * (3 * b + a) : 2 * (3 * a + b);
                const T ur = u[idx], ui = ADJ ? -u[idx + 1] : u[idx + 1];
                const T hr = h[6 * r + 2 * b], hi = h[6 * r + 2 * b + 1];
                re = fmaT(ur, hr, re);
                re = fmaT(-ui, hi, re);
                im = fmaT(ur, hi, im);
                im = fmaT(ui, hr, im);
            }
            w[6 * r + 2 * a] = re;
            w[6 * r + 2 * a + 1] = im;
        }
    }
}

// ---------------------------------------------------------------------------
// FP16-input path (FP16 spinors with FP16 links): v_dot2_f32_f16 forms two
// FP16 products and adds them to an FP32 accumulator, so a complex
// multiply-add is two instructions instead of four FP32 FMAs.  Inputs stay
// in FP16 (the stored spinor and link values; the projected half spinor,
// whose FP16 sum of two FP16 values rounds exactly as the FP32 sum would when
// rounded to FP16; the reconstructed third link row, rounded to FP16);
// products and sums are FP32.
// ---------------------------------------------------------------------------
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

// The two half2 forms of each link element for the dot-product matvec:
//   plain   (u[a][b]):          re = A.h, A = (ur, -ui);  im = B.h, B = (ui, ur)
//   adjoint (conj u[b][a]):     re = A.h, A = (ur,  ui);  im = B.h, B = (-ui, ur)
// indexed [3a + b] for output colour a, input colour b.
template <bool ADJ>
__device__ __forceinline__ void link_forms_f16(const char *U, int cs, int blk, int i, h2_t A[9], h2_t B[9])
{
    const char *p = U + (size_t)blk * 3 * cs * 8;
    const uint32_t off = (uint32_t)i * 8u;
    float u[18];
    _Float16 hv[18];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const half4_t w = ld_off<half4_t, true>(p + (size_t)k * cs * 8, off);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            hv[4 * k + j] = w[j];
            u[4 * k + j] = (float)w[j];
        }
    }
    reconstruct_row3(u);
#pragma unroll
    for (int k = 12; k < 18; k++) hv[k] = (_Float16)u[k];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const int e = ADJ ? 3 * b + a : 3 * a + b;
            const _Float16 ur = hv[2 * e], ui = hv[2 * e + 1];
            if (ADJ) {
                A[3 * a + b] = h2_t{ur, ui};
                B[3 * a + b] = h2_t{-ui, ur};
            } else {
                A[3 * a + b] = h2_t{ur, -ui};
                B[3 * a + b] = h2_t{ui, ur};
            }
        }
}

// (1 + S g_mu) projection on half2 pairs: v[3s + c] = (re, im) of spin s,
// colour c; h[3r + c] for the two independent rows (as project()).
template <int MU, int S>
__device__ __forceinline__ void project_h2(const h2_t v[12], h2_t h[6])
{
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const h2_t p0 = v[c], p1 = v[3 + c], p2 = v[6 + c], p3 = v[9 + c];
        const h2_t ip2 = h2_t{-p2.y, p2.x}, ip3 = h2_t{-p3.y, p3.x};  // i * p
        const _Float16 s = (_Float16)S;
        if (MU == 0) {
            h[c] = p0 + s * ip3;
            h[3 + c] = p1 + s * ip2;
        } else if (MU == 1) {
            h[c] = p0 - s * p3;
            h[3 + c] = p1 + s * p2;
        } else if (MU == 2) {
            h[c] = p0 + s * ip2;
            h[3 + c] = p1 - s * ip3;
        } else {
            h[c] = p0 + s * p2;
            h[3 + c] = p1 + s * p3;
        }
    }
}

// x.lo * y.lo + x.hi * y.hi + 0 in one instruction: the three-operand form
// takes the zero as an inline constant, where the builtin's accumulating
// form would first move a zero into its destination.
__device__ __forceinline__ float dot2_first(h2_t x, h2_t y)
{
    float d;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(d) : "v"(x), "v"(y));
    return d;
}

// w = U h (or U^dag h) for both rows, FP32 results in the float layout of
// su3_mul_half.
__device__ __forceinline__ void su3_mul_half_dot2(const h2_t A[9], const h2_t B[9], const h2_t h[6], float w[12])
{
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            float re = dot2_first(A[3 * a], h[3 * r]), im = dot2_first(B[3 * a], h[3 * r]);
#pragma unroll
            for (int b = 1; b < 3; b++) {
                re = __builtin_amdgcn_fdot2(A[3 * a + b], h[3 * r + b], re, false);
                im = __builtin_amdgcn_fdot2(B[3 * a + b], h[3 * r + b], im, false);
            }
            w[6 * r + 2 * a] = re;
            w[6 * r + 2 * a + 1] = im;
        }
}

// ---------------------------------------------------------------------------
// Block-to-tile mapping.  Work-groups are dispatched round-robin over the
// 8 XCDs (each with its own L2); remapping gives each XCD a contiguous run
// of tiles so that neighbouring lattice slabs share one L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, rm = nb & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + (x < rm ? x : rm) + j;
}


// ---------------------------------------------------------------------------
// Fixed-order reduction of per-site-group partial sums (the CG dot products)
// ---------------------------------------------------------------------------
// A sum of nw partials is formed over kFinLanes virtual lanes: lane v adds
// partials v, v + kFinLanes, v + 2 kFinLanes, ... in that order (loaded four
// at a time; the zeros padding a short last group change no value, at most
// the sign of a zero), then the lanes are combined by a halving tree (lane
// i += lane i + h for h = kFinLanes/2 .. 1).  Every place that finalizes a CG
// scalar uses this order, so the scalars do not depend on where it runs.
constexpr int kFinLanes = 1024;

__device__ __forceinline__ double fin_lane_sum(const double *pp, int nw, int v)
{
    double acc = 0.0;
    for (int w = v; w < nw; w += 4 * kFinLanes) {
        double x[4];
#pragma unroll
        for (int m = 0; m < 4; m++) x[m] = (w + m * kFinLanes < nw) ? pp[w + m * kFinLanes] : 0.0;
#pragma unroll
        for (int m = 0; m < 4; m++) acc += x[m];
    }
    return acc;
}

// Four virtual lanes l + 64 q (q = q0..q3) of one wavefront lane, summed as
// fin_lane_sum does, then paired as the tree pairs them: (q0 + q1) + (q2 + q3).
__device__ __forceinline__ double fin_lanes4(const double *pp, int nw, int l, int q0, int q1, int q2, int q3)
{
    const int qs[4] = {q0, q1, q2, q3};
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w0 = 0; w0 < nw; w0 += 4 * kFinLanes) {
        double x[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const int w = w0 + l + 64 * qs[i] + m * kFinLanes;
                x[i][m] = w < nw ? pp[w] : 0.0;
            }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int m = 0; m < 4; m++) a[i] += x[i][m];
    }
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// The whole sum by one wavefront (lanes l = 0..63 of the calling wave), in
// the order above: virtual lane l + 64 q belongs to lane l, and the tree
// levels h = 512 .. 64 pair q with q + h / 64, i.e. the value of lane l is
// (((s0+s8) + (s4+s12)) + ((s2+s10) + (s6+s14))) + (((s1+s9) + (s5+s13)) +
// ((s3+s11) + (s7+s15))), evaluated four leaves at a time to keep few
// registers live; the last six levels pair lanes.  Result in lane 0.
__device__ __forceinline__ double fin_wave_sum(const double *pp, int nw, int l)
{
    static_assert(kFinLanes == 1024, "the leaf order below is that of 16 virtual lanes per lane");
    const double A = fin_lanes4(pp, nw, l, 0, 8, 4, 12);
    const double B = fin_lanes4(pp, nw, l, 2, 10, 6, 14);
    const double AB = A + B;
    const double C = fin_lanes4(pp, nw, l, 1, 9, 5, 13);
    const double D = fin_lanes4(pp, nw, l, 3, 11, 7, 15);
    double v = AB + (C + D);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_down(v, off, 64);
        if (l < off) v += o;
    }
    return v;
}

// alpha = rr / (p . A p) of CG, with a breakdown (p.Ap <= 0 or not finite)
// poisoning rr; out (may be null) receives a copy of alpha.
__device__ __forceinline__ void fin_alpha_update(double pap, int rid, double *rr, double *alpha, double *out)
{
    if (pap > 0.0 && pap < INFINITY) {
        alpha[rid] = rr[rid] / pap;
    } else {
        alpha[rid] = 0.0;
        rr[rid] = NAN;
    }
    if (out) out[rid] = alpha[rid];
}

}  // namespace wd
