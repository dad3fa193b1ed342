// faces.hip -- the t-faces of a lattice cut along t: what one GPU of a
// t-decomposed lattice sends its two neighbours for each stencil sweep, and
// the boundary update that consumes them.  The paper names running over
// several GPUs as its next step (Sec. 4, end); on one GPU the lattice wraps
// onto itself, so the faces a sweep packs are exactly the ones it would
// receive, and the boundary update can be checked against the stencil.
//
// Sweep with output parity P (input parity Q = 1 - P); S_F = -1 for H and +1
// for H^dag is the sign of the forward projector (1 + S_F g_t), S_B = -S_F:
//   forward face  F[j] = (1 + S_F g_t) psi(y)              y on slice t = 0,
//   backward face B[j] = U_t(y)^dag (1 + S_B g_t) psi(y)   y on slice t = Lt-1,
// each as its two independent spin rows (12 reals, half a spinor); the
// backward face is colour-rotated by the sender, which holds U_t(y).  An
// output site x on slice Lt-1 adds U_t(x) F[j] rebuilt to four spins, one
// on slice 0 adds B[j] rebuilt.  j is the index within the slice: the sites
// of one parity on one t-slice are the contiguous checkerboard range
// [t V3/2, (t+1) V3/2), and x, its t-neighbour across the cut share (x, y, z).
//
// Face layouts (fsp = face sites rounded up to 64): FP64 double2 [6][fsp];
// FP32 float4 [3][fsp]; FP16 the projected values relative to the sending
// site's norm, 4 halves [3][fsp], then that norm, float [fsp].
#include "wd_internal.h"

namespace wd {

namespace {

constexpr int kB = 256;

struct FaceArgs {
    Geom g;
    const char *links;
    const char *in;  // input parity field (parity Q)
    char *out;       // output parity field (parity P)
    char *F;         // forward face
    char *B;         // backward face
    int fs;          // sites of one parity on one t-slice
    int fsp;         // face chunk stride
    int Lt;
    int P;
};

typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

template <int SP> struct HalfIO;

template <> struct HalfIO<SP_F64> {
    static constexpr size_t site_bytes = 96;
    __device__ static void store(char *f, int fsp, int j, const double h[12], float)
    {
        dbl2_t *p = reinterpret_cast<dbl2_t *>(f);
        for (int k = 0; k < 6; k++) p[(size_t)k * fsp + j] = dbl2_t{h[2 * k], h[2 * k + 1]};
    }
    __device__ static float load(const char *f, int fsp, int j, double h[12])
    {
        const dbl2_t *p = reinterpret_cast<const dbl2_t *>(f);
        for (int k = 0; k < 6; k++) {
            const dbl2_t w = p[(size_t)k * fsp + j];
            h[2 * k] = w.x;
            h[2 * k + 1] = w.y;
        }
        return 1.f;
    }
};

template <> struct HalfIO<SP_F32> {
    static constexpr size_t site_bytes = 48;
    __device__ static void store(char *f, int fsp, int j, const float h[12], float)
    {
        flt4_t *p = reinterpret_cast<flt4_t *>(f);
        for (int k = 0; k < 3; k++) p[(size_t)k * fsp + j] = flt4_t{h[4 * k], h[4 * k + 1], h[4 * k + 2], h[4 * k + 3]};
    }
    __device__ static float load(const char *f, int fsp, int j, float h[12])
    {
        const flt4_t *p = reinterpret_cast<const flt4_t *>(f);
        for (int k = 0; k < 3; k++) {
            const flt4_t w = p[(size_t)k * fsp + j];
            h[4 * k] = w.x;
            h[4 * k + 1] = w.y;
            h[4 * k + 2] = w.z;
            h[4 * k + 3] = w.w;
        }
        return 1.f;
    }
};

template <> struct HalfIO<SP_F16> {
    static constexpr size_t site_bytes = 28;
    // h: values relative to the norm n of the sending site
    __device__ static void store(char *f, int fsp, int j, const float h[12], float n)
    {
        u32x2_t *p = reinterpret_cast<u32x2_t *>(f);
        for (int k = 0; k < 3; k++)
            p[(size_t)k * fsp + j] = u32x2_t{cvt_pk_f16(h[4 * k], h[4 * k + 1]), cvt_pk_f16(h[4 * k + 2], h[4 * k + 3])};
        reinterpret_cast<float *>(f + (size_t)24 * fsp)[j] = n;
    }
    __device__ static float load(const char *f, int fsp, int j, float h[12])
    {
        const half4_t *p = reinterpret_cast<const half4_t *>(f);
        for (int k = 0; k < 3; k++) {
            const half4_t w = p[(size_t)k * fsp + j];
            for (int q = 0; q < 4; q++) h[4 * k + q] = (float)w[q];
        }
        return reinterpret_cast<const float *>(f + (size_t)24 * fsp)[j];
    }
};

// The spin projection (1 + S g_t) of the input spinor at checkerboard site
// cb; for FP16 the stored values relative to the site norm n.
template <int SP, int S, typename real>
__device__ __forceinline__ float project_site(const char *in, int cs, int cb, real h[12])
{
    if constexpr (SP == SP_F16) {
        const half8_t *p = reinterpret_cast<const half8_t *>(in);
        _Float16 v[24];
        for (int k = 0; k < 3; k++) {
            const half8_t w = p[(size_t)k * cs + cb];
            for (int q = 0; q < 8; q++) v[8 * k + q] = w[q];
        }
        project_mix<3, S>(v, h);
        return reinterpret_cast<const float *>(in + (size_t)48 * cs)[cb];
    } else {
        real v[24];
        SpinorIO<SP>::load(in, cs, cb, v);
        project<3, S>(v, h);
        return 1.f;
    }
}

template <int SP, int LK, bool DAG>
__global__ void __launch_bounds__(kB) k_pack_faces(FaceArgs a)
{
    typedef typename SpinorIO<SP>::real real;
    constexpr int SF = DAG ? +1 : -1, SB = -SF;
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= 2 * a.fs) return;
    const int cs = a.g.cs;
    real h[12];
    if (i < a.fs) {
        const float n = project_site<SP, SF>(a.in, cs, i, h);
        HalfIO<SP>::store(a.F, a.fsp, i, h, n);
    } else {
        const int j = i - a.fs;
        const int cb = (a.Lt - 1) * a.fs + j;
        const float n = project_site<SP, SB>(a.in, cs, cb, h);
        real u[18], w[12];
        LinkIO<LK>::load(a.links, cs, (1 - a.P) * 4 + 3, cb, u);
        su3_mul_half<true>(u, h, w);
        HalfIO<SP>::store(a.B, a.fsp, j, w, n);
    }
}

template <int SP, int LK, bool DAG>
__global__ void __launch_bounds__(kB) k_apply_faces(FaceArgs a)
{
    typedef typename SpinorIO<SP>::real real;
    constexpr int SF = DAG ? +1 : -1, SB = -SF;
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= 2 * a.fs) return;
    const int cs = a.g.cs;
    real acc[24], w[12];
    if (i < a.fs) {  // output slice Lt-1: forward neighbour across the cut
        const int cb = (a.Lt - 1) * a.fs + i;
        real h[12], u[18];
        const real n = (real)HalfIO<SP>::load(a.F, a.fsp, i, h);
        LinkIO<LK>::load(a.links, cs, a.P * 4 + 3, cb, u);
        su3_mul_half<false>(u, h, w);
        SpinorIO<SP>::load(a.out, cs, cb, acc);
        if constexpr (has_norm(SP))
            accumulate_scaled<3, SF>(acc, w, n);
        else
            accumulate<3, SF>(acc, w);
        SpinorIO<SP>::store(a.out, cs, cb, acc);
    } else {  // output slice 0: backward neighbour across the cut
        const int cb = i - a.fs;
        const real n = (real)HalfIO<SP>::load(a.B, a.fsp, cb, w);
        SpinorIO<SP>::load(a.out, cs, cb, acc);
        if constexpr (has_norm(SP))
            accumulate_scaled<3, SB>(acc, w, n);
        else
            accumulate<3, SB>(acc, w);
        SpinorIO<SP>::store(a.out, cs, cb, acc);
    }
}

size_t face_site_bytes(int sp)
{
    return sp == SP_F64 ? HalfIO<SP_F64>::site_bytes : (sp == SP_F32 ? HalfIO<SP_F32>::site_bytes : HalfIO<SP_F16>::site_bytes);
}

// The spinor / link precision pairs the solver uses (see decode_prec).
#define WD_FACE_PAIRS(X)                                                                          \
    X(SP_F64, LK_F64_18) X(SP_F64, LK_F64_12) X(SP_F32, LK_F32_12) X(SP_F32, LK_F32_18)           \
    X(SP_F32, LK_F16_12) X(SP_F16, LK_F32_12) X(SP_F16, LK_F32_18) X(SP_F16, LK_F16_12)

hipError_t launch_faces(bool pack, int sp, int lk, int dag, const FaceArgs &a, hipStream_t s)
{
    const dim3 grid((2 * a.fs + kB - 1) / kB);
#define X(SP_, LK_)                                                                               \
    if (sp == SP_ && lk == LK_) {                                                                 \
        if (pack) {                                                                               \
            if (dag) hipLaunchKernelGGL((k_pack_faces<SP_, LK_, true>), grid, dim3(kB), 0, s, a);  \
            else hipLaunchKernelGGL((k_pack_faces<SP_, LK_, false>), grid, dim3(kB), 0, s, a);    \
        } else {                                                                                  \
            if (dag) hipLaunchKernelGGL((k_apply_faces<SP_, LK_, true>), grid, dim3(kB), 0, s, a); \
            else hipLaunchKernelGGL((k_apply_faces<SP_, LK_, false>), grid, dim3(kB), 0, s, a);   \
        }                                                                                         \
        return hipGetLastError();                                                                 \
    }
    WD_FACE_PAIRS(X)
#undef X
    return hipErrorInvalidValue;
}

// Context fields and faces for one sweep of output parity P.
wd_status face_setup(wd_ctx *c, int prec, int P, int *sp, int *lk, Field *fi, Field *fo, FaceArgs *a)
{
    int xp;
    WD_TRY(decode_prec(c, prec, sp, lk, &xp));
    if (*sp == SP_I16) return set_error(WD_ERR_ARG, "faces take FP64, FP32 or FP16 spinors");
    if (*lk == LK_F32_8) return set_error(WD_ERR_ARG, "faces take 12- or 18-real links");
    WD_TRY(alloc_field(c, "fc_in", *sp, 1, 1, fi));
    WD_TRY(alloc_field(c, "fc_out", *sp, 1, 1, fo));
    const int fs = c->g.Lxh * c->g.L[1] * c->g.L[2];
    const int fsp = (fs + 63) / 64 * 64;
    const size_t fb = face_site_bytes(*sp) * (size_t)fsp;
    void *buf;
    WD_TRY(ws_get(c, "fc_faces", 2 * fb, &buf));
    a->g = c->g;
    a->links = link_ptr(c, *lk);
    a->in = fi->base;
    a->out = fo->base;
    a->F = (char *)buf;
    a->B = (char *)buf + fb;
    a->fs = fs;
    a->fsp = fsp;
    a->Lt = c->g.L[3];
    a->P = P;
    return WD_OK;
}

}  // namespace

}  // namespace wd

using namespace wd;

extern "C" wd_status wd_faces_apply(wd_ctx *c, double *out, const double *in, int out_parity, int dagger,
                                    int prec)
{
    if (!c || !out || !in) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    if (out_parity != WD_EVEN && out_parity != WD_ODD)
        return set_error(WD_ERR_ARG, "output parity %d is not WD_EVEN or WD_ODD", out_parity);
    WD_HIP(hipSetDevice(c->device));
    const int P = (out_parity == WD_EVEN) ? 0 : 1;
    int sp, lk;
    Field fi, fo;
    FaceArgs a;
    WD_TRY(face_setup(c, prec, P, &sp, &lk, &fi, &fo, &a));
    hipStream_t s = c->stream;
    hipError_t e;
    if ((e = pack_spinor(in, fi, 1, 0, c->g, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
    WD_HIP(hipMemsetAsync(fo.base, 0, (size_t)fo.rs, s));
    if ((e = launch_faces(true, sp, lk, dagger, a, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "face pack: %s", hipGetErrorString(e));
    if ((e = launch_faces(false, sp, lk, dagger, a, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "face update: %s", hipGetErrorString(e));
    if ((e = unpack_spinor(fo, out, 1, 0, c->g, s)) != hipSuccess)
        return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    return WD_OK;
}

extern "C" wd_status wd_bench_faces(wd_ctx *c, int prec, int iters, double *pack_ms, double *apply_ms,
                                    double *pack_bytes, double *apply_bytes)
{
    if (!c || !pack_ms || !apply_ms) return set_error(WD_ERR_ARG, "NULL argument");
    if (iters < 1) return set_error(WD_ERR_ARG, "iters %d < 1", iters);
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    WD_HIP(hipSetDevice(c->device));
    int sp, lk;
    Field fi, fo;
    FaceArgs a;
    WD_TRY(face_setup(c, prec, 0, &sp, &lk, &fi, &fo, &a));
    hipStream_t s = c->stream;
    WD_HIP(hipMemsetAsync(fi.base, 0, (size_t)fi.rs, s));
    WD_HIP(hipMemsetAsync(fo.base, 0, (size_t)fo.rs, s));
    hipEvent_t e0, e1, e2;
    WD_HIP(hipEventCreate(&e0));
    WD_HIP(hipEventCreate(&e1));
    WD_HIP(hipEventCreate(&e2));
    hipError_t e = launch_faces(true, sp, lk, 0, a, s);
    if (e == hipSuccess) e = launch_faces(false, sp, lk, 0, a, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int it = 0; it < iters && e == hipSuccess; it++) e = launch_faces(true, sp, lk, 0, a, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    for (int it = 0; it < iters && e == hipSuccess; it++) e = launch_faces(false, sp, lk, 0, a, s);
    if (e == hipSuccess) e = hipEventRecord(e2, s);
    if (e == hipSuccess) e = hipEventSynchronize(e2);
    float t1 = 0, t2 = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t1, e0, e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t2, e1, e2);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    if (e != hipSuccess) return set_error(WD_ERR_HIP, "face benchmark: %s", hipGetErrorString(e));
    *pack_ms = t1 / iters;
    *apply_ms = t2 / iters;
    // bytes each sweep must move: pack reads both input slices and the
    // backward links and writes both faces; the update reads the faces, the
    // forward links and both output slices, and writes the output slices
    const double fsb = (double)a.fs, sb = (double)spinor_site_bytes(sp), lb = (double)link_bytes(lk);
    const double hb = (double)face_site_bytes(sp);
    if (pack_bytes) *pack_bytes = fsb * (2 * sb + lb + 2 * hb);
    if (apply_bytes) *apply_bytes = fsb * (2 * hb + lb + 4 * sb);
    return WD_OK;
}
