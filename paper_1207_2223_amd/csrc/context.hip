// context.hip -- context lifetime, gauge-field loading, the stencil launcher
// with optional event timing, and the operator-level C-ABI calls
// (wd_dslash, wd_mdagm, index tables).
#include <stdarg.h>
#include <stdio.h>

#include <cmath>
#include <cstring>
#include <tuple>

#include "wd_internal.h"

namespace wd {

static thread_local char g_err[512] = "no error";

wd_status set_error(wd_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

wd_status ws_get(wd_ctx *c, const std::string &name, size_t bytes, void **ptr)
{
    auto it = c->ws.find(name);
    if (it != c->ws.end() && it->second.second >= bytes) {
        *ptr = it->second.first;
        return WD_OK;
    }
    if (it != c->ws.end()) {
        WD_HIP(hipStreamSynchronize(c->stream));
        WD_HIP(hipFree(it->second.first));
        c->ws.erase(it);
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(WD_ERR_OOM, "device allocation of %zu bytes for '%s' failed", bytes,
                         name.c_str());
    }
    c->ws[name] = {p, bytes};
    *ptr = p;
    return WD_OK;
}

wd_status pinned_get(wd_ctx *c, int slot, size_t bytes, void **ptr)
{
    if (c->pinned_bytes[slot] < bytes) {
        if (c->pinned[slot]) {
            WD_HIP(hipStreamSynchronize(c->stream));
            WD_HIP(hipHostFree(c->pinned[slot]));
            c->pinned[slot] = nullptr;
        }
        size_t nb = bytes < 4096 ? 4096 : bytes;
        WD_HIP(hipHostMalloc(&c->pinned[slot], nb, hipHostMallocDefault));
        c->pinned_bytes[slot] = nb;
    }
    *ptr = c->pinned[slot];
    return WD_OK;
}

wd_status alloc_field(wd_ctx *c, const std::string &name, int sp, int nsub, int nrhs, Field *f)
{
    const long long sb = (long long)spinor_site_bytes(sp) * c->g.cs;
    const long long sub = (sb + 255) / 256 * 256;
    void *p = nullptr;
    WD_TRY(ws_get(c, name, (size_t)sub * nsub * nrhs, &p));
    f->base = (char *)p;
    f->ss = sub;
    f->rs = sub * nsub;
    f->sp = sp;
    f->nsub = nsub;
    f->cs = c->g.cs;
    return WD_OK;
}

const char *link_ptr(const wd_ctx *c, int lk)
{
    if (lk == LK_F64_18 || lk == LK_F64_12) return c->links64;
    if (lk == LK_F32_12) return c->links32;
    if (lk == LK_F32_18) return c->links32r;
    if (lk == LK_F32_8) return c->links8;
    return c->links16;
}

wd_status decode_prec(const wd_ctx *c, int prec, int *sp, int *lk, int *xp)
{
    const int base = prec & 0xf;
    const bool l16 = (prec & WD_LINKS_F16) != 0, r18 = (prec & WD_LINKS_R18) != 0, r8 = (prec & WD_LINKS_R8) != 0;
    if ((prec & ~(0xf | WD_LINKS_F16 | WD_LINKS_R18 | WD_LINKS_R8)) || base > WD_I16 ||
        (base == WD_F64 && (l16 || r18 || r8)) || (int)l16 + (int)r18 + (int)r8 > 1 ||
        (base == WD_I16 && (r18 || r8)))
        return set_error(WD_ERR_ARG, "bad precision code 0x%x", prec);
    *sp = base == WD_F64 ? SP_F64 : (base == WD_F32 ? SP_F32 : (base == WD_F16 ? SP_F16 : SP_I16));
    *lk = *sp == SP_F64 ? c->lk64 : (l16 ? LK_F16_12 : (r18 ? LK_F32_18 : (r8 ? LK_F32_8 : LK_F32_12)));
    *xp = *sp == SP_F64 ? SP_F64 : SP_F32;
    return WD_OK;
}

TuneCfg default_cfg(int sp)
{
    TuneCfg t;
    t.block = 128;
    t.nr = 1;
    t.rl = 1;
    t.remap = 1;
    (void)sp;
    return t;
}

double sweep_bytes(const wd_ctx *c, const Sweep &sw)
{
    const double sb = (double)spinor_site_bytes(sw.sp);
    // each field read or written once: plain in, out; xpay in, x, out; CG
    // update in, x, r read and written
    double per_rhs = 2 * sb;
    if (sw.epi == EPI_XPAY) per_rhs = 3 * sb;
    if (sw.epi == EPI_CGUPD) per_rhs = 4 * sb;
    return (double)c->Vh * (8.0 * (double)link_bytes(sw.lk) + sw.nact * per_rhs);
}

// Per-launch HIP events of the stencil timing (wd_timing_enable).
static wd_status timing_begin(wd_ctx *c, hipEvent_t *e0, hipEvent_t *e1)
{
    if (c->ev_used == c->events.size()) {
        hipEvent_t x0, x1;
        WD_HIP(hipEventCreate(&x0));
        WD_HIP(hipEventCreate(&x1));
        c->events.push_back({x0, x1});
    }
    *e0 = c->events[c->ev_used].first;
    *e1 = c->events[c->ev_used].second;
    c->ev_used++;
    WD_HIP(hipEventRecord(*e0, c->stream));
    return WD_OK;
}

// kind: 0 dslash_kernel, 1 dslash_lds_kernel, 2 dslash_tw_kernel
static void timing_end(wd_ctx *c, const Sweep &sw, hipEvent_t e1, int kind, int nr, int rl, int lk)
{
    (void)hipEventRecord(e1, c->stream);
    const double b = sweep_bytes(c, sw);
    char name[96];
    // the kernel's template instance as profilers print it
    if (kind != 0)
        snprintf(name, sizeof(name), "dslash_%s_kernel<%d, %d, %d, %s, %d>", kind == 1 ? "lds" : "tw", sw.sp,
                 sw.lk, nr, sw.dag ? "true" : "false", sw.epi);
    else
        snprintf(name, sizeof(name), "dslash_kernel<%d, %d, %d, %d, %s, %d>", sw.sp, lk, nr, rl,
                 sw.dag ? "true" : "false", sw.epi);
    if (c->ev_info.size() < c->ev_used) c->ev_info.resize(c->ev_used);
    c->ev_info[c->ev_used - 1] = std::make_tuple(std::string(name), b, (double)c->Vh * sw.nact);
    c->t_bytes += b;
    c->t_launches++;
}

wd_status run_sweep(wd_ctx *c, const Sweep &sw, const TuneCfg *cfg)
{
    if (sw.nact <= 0) return WD_OK;
    if (!cfg && c->use_tuned) cfg = tuned_cfg(c, sw);
    TuneCfg t = cfg ? *cfg : default_cfg(sw.sp);
    if (!dslash_shape_supported(sw.sp, sw.lk, t.nr, t.rl) || t.block < 64 || t.block > 256 || (t.block & 63))
        return set_error(WD_ERR_ARG, "unsupported launch shape block %d nr %d rl %d", t.block, t.nr, t.rl);
    if (t.lnt != 0 && (t.lnt != 1 || !lnt_ok(sw.sp, sw.lk, t)))
        return set_error(WD_ERR_ARG, "non-temporal links need FP32 12- or 8-real or FP64 12-real links, the "
                         "register-tiled kernel, 1 lane per site and 1 or 2 RHS per lane (block %d nr %d rl %d "
                         "order %d)", t.block, t.nr, t.rl, t.remap);
    const int nr = t.nr, rl = t.rl;
    DslashArgs a;
    a.g = c->g;
    a.P = sw.P;
    a.links = sw.links ? sw.links : link_ptr(c, sw.lk);
    a.in = sw.in.base;
    a.in_rs = sw.in.rs;
    a.out = sw.out.base;
    a.out_rs = sw.out.rs;
    a.x = sw.x.base;
    a.x_rs = sw.x.rs;
    a.coef = sw.coef;
    a.r = sw.r.base;
    a.r_rs = sw.r.rs;
    a.alpha = sw.alpha;
    a.active = sw.active;
    a.nact = sw.nact;
    a.G = (sw.nact + nr * rl - 1) / (nr * rl);
    a.remap = t.remap;
    a.partial = sw.partial;
    a.pstride = sw.pstride;
    a.pw_off = sw.pw_off;
    a.fin_blocks = sw.fin_partial ? sw.nact : 0;
    a.fin_nw = sw.fin_nw;
    a.fin_pstride = sw.fin_pstride;
    a.fin_partial = sw.fin_partial;
    a.fin_rr = sw.fin_rr;
    a.fin_alpha = sw.fin_alpha;
    a.fin_out = sw.fin_out;
    if (t.occ != 0 && (t.occ < 2 || t.occ > kMaxOcc))
        return set_error(WD_ERR_ARG, "work-group cap %d not 0 or in 2..%d", t.occ, kMaxOcc);
    a.lds = occ_lds_bytes(t.occ);
    const int spb = t.block / rl;
    const int ntiles = (int)((c->Vh + spb - 1) / spb);
    a.tpp = 1;
    a.nzl = 1;
    a.nys = 1;
    a.tch = 1;
    if (is_tw_order(t.remap)) {
        if (!tw_order_ok(c, sw.sp, sw.lk, nr, rl, t.block, t.remap))
            return set_error(WD_ERR_ARG, "t-walking order %d does not apply here (sp %d lk %d nr %d rl %d block %d)",
                             t.remap, sw.sp, sw.lk, nr, rl, t.block);
        a.tpp = c->g.Lxh * c->g.L[1] / t.block;
        a.nzl = c->g.L[2] / 8;
        a.tch = tw_chunk(t.remap);
        const long long grid = (long long)c->g.L[2] * a.tpp * a.G * (c->g.L[3] / a.tch) + a.fin_blocks;
        if (grid > 0x7fffffffLL) return set_error(WD_ERR_ARG, "grid too large");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) WD_TRY(timing_begin(c, &e0, &e1));
        hipError_t e = dslash_tw_launch(a, sw.sp, sw.lk, nr, sw.dag, sw.epi, t.block, (int)grid, c->stream);
        if (e != hipSuccess)
            return set_error(WD_ERR_HIP, "t-walking stencil launch (sp %d lk %d nr %d epi %d block %d): %s", sw.sp,
                             sw.lk, nr, sw.epi, t.block, hipGetErrorString(e));
        if (c->timing) timing_end(c, sw, e1, 2, nr, rl, sw.lk);
        return WD_OK;
    }
    if (is_lds_order(t.remap)) {
        if (!lds_order_ok(c, sw.sp, sw.lk, nr, t.remap) || rl != 1 || t.block != 256 || t.occ != 0)
            return set_error(WD_ERR_ARG, "LDS-staged order %d does not apply here (sp %d lk %d nr %d rl %d block %d "
                             "cap %d)", t.remap, sw.sp, sw.lk, nr, rl, t.block, t.occ);
        a.tpp = lds_chunk(t.remap);
        a.nzl = c->g.L[2] / 8;
        a.lds = lds_order_bytes(c, sw.sp, nr);
        const long long grid = (long long)c->g.L[2] * (c->g.L[3] / a.tpp) * a.G + a.fin_blocks;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) WD_TRY(timing_begin(c, &e0, &e1));
        hipError_t e = dslash_lds_launch(a, sw.sp, sw.lk, nr, sw.dag, sw.epi, (int)grid, a.lds, c->stream);
        if (e != hipSuccess)
            return set_error(WD_ERR_HIP, "LDS stencil launch (sp %d lk %d nr %d epi %d, %u bytes LDS): %s", sw.sp,
                             sw.lk, nr, sw.epi, a.lds, hipGetErrorString(e));
        if (c->timing) timing_end(c, sw, e1, 1, nr, rl, sw.lk);
        return WD_OK;
    }
    if (t.remap >= kTileOrders || t.remap < 0) return set_error(WD_ERR_ARG, "tile order %d unknown", t.remap);
    if (t.remap >= 2) {
        if (!slab_order_ok(c->g, spb, t.remap))
            return set_error(WD_ERR_ARG, "slab tile order %d needs Lz (or Lt) %% 8 == 0 and whole tiles per "
                             "plane and stripe", t.remap);
        a.tpp = c->g.Lxh * c->g.L[1] / spb;
        a.nzl = c->g.L[remap_slab_dim(t.remap)] / 8;
        a.nys = remap_stripes(t.remap);
    }
    const long long grid = (long long)ntiles * a.G + a.fin_blocks;
    if (grid > 0x7fffffffLL) return set_error(WD_ERR_ARG, "grid too large");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) WD_TRY(timing_begin(c, &e0, &e1));
    // (non-temporal links: the same packed field, read by the LK_F32_12N instance)
    const int lk_run = t.lnt ? lnt_variant(sw.lk) : sw.lk;
    hipError_t e = dslash_launch(a, sw.sp, lk_run, nr, rl, sw.dag, sw.epi, t.block, (int)grid, c->stream);
    if (e != hipSuccess)
        return set_error(WD_ERR_HIP, "stencil launch (sp %d lk %d nr %d rl %d epi %d block %d): %s",
                         sw.sp, lk_run, nr, rl, sw.epi, t.block, hipGetErrorString(e));
    if (c->timing) timing_end(c, sw, e1, 0, nr, rl, lk_run);
    return WD_OK;
}

unsigned lds_order_bytes(const wd_ctx *c, int sp, int nr)
{
    return 3u * (unsigned)nr * (unsigned)(c->g.Lxh * c->g.L[1]) * (unsigned)spinor_site_bytes(sp);
}

bool lds_order_ok(const wd_ctx *c, int sp, int lk, int nr, int remap)
{
    if (!is_lds_order(remap) || !dslash_lds_supported(sp, lk, nr)) return false;
    const int S = c->g.Lxh * c->g.L[1];
    return S % 64 == 0 && S <= 512 && c->g.L[2] % 8 == 0 && c->g.L[3] % lds_chunk(remap) == 0 &&
           (long long)lds_order_bytes(c, sp, nr) <= (long long)c->lds_max;
}

bool lnt_ok(int sp, int lk, const TuneCfg &t)
{
    const bool fmt = (lk == LK_F64_12) ? sp == SP_F64
                                       : ((lk == LK_F32_12 || lk == LK_F32_8) && (sp == SP_F16 || sp == SP_F32));
    return fmt && t.rl == 1 && (t.nr == 1 || t.nr == 2) && t.remap >= 0 && t.remap < kTileOrders;
}

bool tw_order_ok(const wd_ctx *c, int sp, int lk, int nr, int rl, int block, int remap)
{
    if (!is_tw_order(remap) || !dslash_tw_supported(sp, lk, nr) || rl != 1) return false;
    const int S = c->g.Lxh * c->g.L[1];
    return (block == 64 || block == 128 || block == 256) && S % block == 0 && c->g.L[2] % 8 == 0 &&
           c->g.L[3] % tw_chunk(remap) == 0;
}

bool slab_order_ok(const Geom &g, int spb, int remap)
{
    const int plane = g.Lxh * g.L[1];
    if (g.L[remap_slab_dim(remap)] % 8 != 0 || spb <= 0 || plane % spb != 0) return false;
    return (plane / spb) % remap_stripes(remap) == 0;
}

static wd_status upload(wd_ctx *c, void *dst, const void *src, size_t bytes)
{
    void *h = nullptr;
    WD_HIP(hipStreamSynchronize(c->stream));
    WD_TRY(pinned_get(c, 0, bytes, &h));
    std::memcpy(h, src, bytes);
    WD_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, c->stream));
    WD_HIP(hipStreamSynchronize(c->stream));
    return WD_OK;
}

wd_status upload_doubles(wd_ctx *c, const std::string &name, const double *v, int n, double **dev)
{
    void *p = nullptr;
    WD_TRY(ws_get(c, name, sizeof(double) * n, &p));
    WD_TRY(upload(c, p, v, sizeof(double) * n));
    *dev = (double *)p;
    return WD_OK;
}

wd_status upload_ints(wd_ctx *c, const std::string &name, const int *v, int n, int **dev)
{
    void *p = nullptr;
    WD_TRY(ws_get(c, name, sizeof(int) * (n ? n : 1), &p));
    if (n) WD_TRY(upload(c, p, v, sizeof(int) * n));
    *dev = (int *)p;
    return WD_OK;
}

Field sub_view(const Field &f, int s)
{
    Field v = f;
    v.base = f.base + s * f.ss;
    v.nsub = 1;
    v.ss = 0;
    return v;
}

}  // namespace wd

using namespace wd;

extern "C" {

const char *wd_last_error(void) { return g_err; }

const char *wd_version(void) { return "wd 0.1 (gfx950)"; }

void wd_solver_defaults(wd_solver_params *p)
{
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 20000;
    p->prec_sloppy = WD_F64;
    p->eo = 1;
    p->delta = 0.1;
    p->poll = 8;
    p->tuned = 0;
    p->graphs = 1;
    p->initial_guess = 0;
}

static wd_status check_dims(const int32_t *dims, long long *V)
{
    if (!dims) return set_error(WD_ERR_ARG, "dims is NULL");
    long long v = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (dims[mu] < 2 || (dims[mu] & 1))
            return set_error(WD_ERR_DIMS, "extent %d of direction %d must be even and >= 2", dims[mu], mu);
        v *= dims[mu];
    }
    if (v >= (1LL << 31)) return set_error(WD_ERR_DIMS, "volume %lld too large", v);
    // the stencil addresses one chunk array (16-byte elements, one parity) with
    // 32-bit byte offsets
    if ((long long)padded_stride((int)(v / 2)) * 16 > 0xFFFFFFFFLL)
        return set_error(WD_ERR_DIMS, "volume %lld too large: one parity's chunk array must stay below 4 GiB", v);
    *V = v;
    return WD_OK;
}

wd_status wd_create(wd_ctx **out, const int32_t dims[4], int device, void *hip_stream)
{
    if (!out) return set_error(WD_ERR_ARG, "NULL context pointer");
    long long V;
    WD_TRY(check_dims(dims, &V));
    int ndev = 0;
    WD_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(WD_ERR_ARG, "device %d not present", device);
    WD_HIP(hipSetDevice(device));
    WD_TRY(scratch_setup(device));
    int lds_max = 0;
    WD_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    wd_ctx *c = new wd_ctx();
    c->device = device;
    c->lds_max = lds_max;
    c->stream = (hipStream_t)hip_stream;
    for (int mu = 0; mu < 4; mu++) {
        c->dims[mu] = dims[mu];
        c->g.L[mu] = dims[mu];
    }
    c->V = V;
    c->Vh = V / 2;
    c->g.Vh = (int)c->Vh;
    c->g.Lxh = dims[0] / 2;
    c->g.sy = c->g.Lxh;
    c->g.sz = c->g.Lxh * dims[1];
    c->g.st = c->g.Lxh * dims[1] * dims[2];
    c->g.cs = padded_stride((int)c->Vh);
    c->g.dxh = make_fastdiv(c->g.Lxh);
    c->g.dy = make_fastdiv(dims[1]);
    c->g.dz = make_fastdiv(dims[2]);
    *out = c;
    return WD_OK;
}

wd_status wd_destroy(wd_ctx *c)
{
    if (!c) return WD_OK;
    if (c->sessions > 0)
        return set_error(WD_ERR_STATE, "%d solver session(s) still open on this context: destroy them first",
                         c->sessions);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->ws) (void)hipFree(kv.second.first);
    if (c->links64) (void)hipFree(c->links64);
    if (c->links32) (void)hipFree(c->links32);
    if (c->links16) (void)hipFree(c->links16);
    if (c->links32r) (void)hipFree(c->links32r);
    if (c->links8) (void)hipFree(c->links8);
    for (int k = 0; k < 2; k++)
        if (c->pinned[k]) (void)hipHostFree(c->pinned[k]);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
    return WD_OK;
}

wd_status wd_set_stream(wd_ctx *c, void *hip_stream)
{
    if (!c) return set_error(WD_ERR_ARG, "NULL context");
    WD_HIP(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)hip_stream;
    return WD_OK;
}

wd_status wd_gauge_load(wd_ctx *c, const double *U, uint32_t flags)
{
    if (!c || !U) return set_error(WD_ERR_ARG, "NULL argument");
    if (flags & ~1u) return set_error(WD_ERR_ARG, "unknown gauge flags 0x%x", flags);
    WD_HIP(hipSetDevice(c->device));
    const int lk64 = (flags & WD_RECON_12) ? LK_F64_12 : LK_F64_18;
    const size_t nl = (size_t)8 * c->g.cs;  // (parity, mu) blocks of cs link slots
    const size_t n64 = link_bytes(lk64) * nl, n32 = link_bytes(LK_F32_12) * nl,
                 n16 = link_bytes(LK_F16_12) * nl, n32r = link_bytes(LK_F32_18) * nl,
                 n8 = link_bytes(LK_F32_8) * nl;
    WD_HIP(hipStreamSynchronize(c->stream));
    if (c->links64 && c->lk64 != lk64) {
        WD_HIP(hipFree(c->links64));
        c->links64 = nullptr;
    }
    auto alloc = [&](char **p, size_t n) -> wd_status {
        if (*p) return WD_OK;
        if (hipMalloc((void **)p, n) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return set_error(WD_ERR_OOM, "gauge allocation of %zu bytes failed", n);
        }
        return WD_OK;
    };
    WD_TRY(alloc(&c->links64, n64));
    WD_TRY(alloc(&c->links32, n32));
    WD_TRY(alloc(&c->links16, n16));
    WD_TRY(alloc(&c->links32r, n32r));
    WD_TRY(alloc(&c->links8, n8));
    c->lk64 = lk64;
    hipError_t e;
    if ((e = pack_gauge(U, c->links64, lk64, c->g, c->stream)) != hipSuccess ||
        (e = pack_gauge(U, c->links32, LK_F32_12, c->g, c->stream)) != hipSuccess ||
        (e = pack_gauge(U, c->links16, LK_F16_12, c->g, c->stream)) != hipSuccess ||
        (e = pack_gauge(U, c->links32r, LK_F32_18, c->g, c->stream)) != hipSuccess ||
        (e = pack_gauge(U, c->links8, LK_F32_8, c->g, c->stream)) != hipSuccess)
        return set_error(WD_ERR_HIP, "gauge packing failed: %s", hipGetErrorString(e));
    c->have_gauge = true;
    return WD_OK;
}


wd_status wd_dslash(wd_ctx *c, double *out, const double *in, int out_parity, int dagger, int prec)
{
    if (!c || !out || !in) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    if (out_parity < WD_FULL || out_parity > WD_ODD) return set_error(WD_ERR_ARG, "bad parity %d", out_parity);
    int sp, lk, xp;
    WD_TRY(decode_prec(c, prec, &sp, &lk, &xp));
    WD_HIP(hipSetDevice(c->device));
    const int full = (out_parity == WD_FULL);
    Field fi, fo;
    WD_TRY(alloc_field(c, "dsl_in", sp, 2, 1, &fi));
    WD_TRY(alloc_field(c, "dsl_out", sp, 2, 1, &fo));
    int zero = 0;
    int *act;
    WD_TRY(upload_ints(c, "dsl_act", &zero, 1, &act));
    hipError_t e;
    if (full) {
        if ((e = pack_spinor(in, fi, 1, 1, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
        for (int P = 0; P < 2; P++) {
            Sweep sw;
            sw.sp = sp; sw.lk = lk; sw.dag = dagger ? 1 : 0; sw.epi = EPI_PLAIN; sw.P = P;
            sw.in = sub_view(fi, 1 - P);
            sw.out = sub_view(fo, P);
            sw.active = act; sw.nact = 1;
            WD_TRY(run_sweep(c, sw, nullptr));
        }
        if ((e = unpack_spinor(fo, out, 1, 1, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    } else {
        const int P = (out_parity == WD_EVEN) ? 0 : 1;
        Field vi = sub_view(fi, 0), vo = sub_view(fo, 0);
        if ((e = pack_spinor(in, vi, 1, 0, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
        Sweep sw;
        sw.sp = sp; sw.lk = lk; sw.dag = dagger ? 1 : 0; sw.epi = EPI_PLAIN; sw.P = P;
        sw.in = vi; sw.out = vo; sw.active = act; sw.nact = 1;
        WD_TRY(run_sweep(c, sw, nullptr));
        if ((e = unpack_spinor(vo, out, 1, 0, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    }
    return WD_OK;
}

namespace {
__global__ void __launch_bounds__(256) k_fill_ones(unsigned *p, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0xffffffffu;
}

hipError_t fill_ones(void *p, size_t bytes, hipStream_t s)
{
    const long long n = (long long)(bytes / 4);
    if (n > 0)
        hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (unsigned *)p, n);
    return hipGetLastError();
}
}  // namespace

wd_status wd_dslash_shaped(wd_ctx *c, double *out, const double *in, int nrhs, int out_parity, int dagger,
                           int prec, const int32_t shape[5])
{
    if (!c || !out || !in) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    if (out_parity != WD_EVEN && out_parity != WD_ODD)
        return set_error(WD_ERR_ARG, "bad parity %d (WD_EVEN or WD_ODD)", out_parity);
    if (nrhs < 1 || nrhs > 64) return set_error(WD_ERR_ARG, "nrhs %d out of range 1..64", nrhs);
    int sp, lk, xp;
    WD_TRY(decode_prec(c, prec, &sp, &lk, &xp));
    TuneCfg t = default_cfg(sp);
    if (shape) {
        t.block = shape[0];
        t.nr = shape[1];
        t.rl = shape[2];
        t.remap = shape[3];
        t.occ = shape[4];
    }
    const bool lds_ok = (is_lds_order(t.remap) && lds_order_ok(c, sp, lk, t.nr, t.remap) && t.rl == 1 &&
                         t.block == 256 && t.occ == 0) ||
                        (is_tw_order(t.remap) && tw_order_ok(c, sp, lk, t.nr, t.rl, t.block, t.remap) &&
                         (t.occ == 0 || (t.occ >= 2 && t.occ <= kMaxOcc)));
    if (!lds_ok && (!dslash_shape_supported(sp, lk, t.nr, t.rl) || t.block < 64 || t.block > 256 || (t.block & 63) ||
                    t.remap < 0 || t.remap >= kTileOrders || (t.occ != 0 && (t.occ < 2 || t.occ > kMaxOcc)) ||
                    (t.remap >= 2 && !slab_order_ok(c->g, t.block / t.rl, t.remap))))
        return set_error(WD_ERR_ARG, "launch shape block %d nr %d rl %d order %d cap %d not supported here",
                         t.block, t.nr, t.rl, t.remap, t.occ);
    WD_HIP(hipSetDevice(c->device));
    Field fi, fo;
    WD_TRY(alloc_field(c, "dsh_in", sp, 1, nrhs, &fi));
    WD_TRY(alloc_field(c, "dsh_out", sp, 1, nrhs, &fo));
    std::vector<int> ids(nrhs);
    for (int j = 0; j < nrhs; j++) ids[j] = j;
    int *act;
    WD_TRY(upload_ints(c, "dsh_act", ids.data(), nrhs, &act));
    hipError_t e;
    if ((e = pack_spinor(in, fi, nrhs, 0, c->g, c->stream)) != hipSuccess)
        return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
    // poison the internal output (all-ones bytes: NaN in every format), so
    // that sites a launch shape failed to write show up as NaN
    if ((e = fill_ones(fo.base, (size_t)fo.rs * nrhs, c->stream)) != hipSuccess)
        return set_error(WD_ERR_HIP, "fill: %s", hipGetErrorString(e));
    Sweep sw;
    sw.sp = sp; sw.lk = lk; sw.dag = dagger ? 1 : 0; sw.epi = EPI_PLAIN;
    sw.P = (out_parity == WD_EVEN) ? 0 : 1;
    sw.in = fi; sw.out = fo; sw.active = act; sw.nact = nrhs;
    WD_TRY(run_sweep(c, sw, &t));
    if ((e = unpack_spinor(fo, out, nrhs, 0, c->g, c->stream)) != hipSuccess)
        return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    return WD_OK;
}

extern "C++" {
namespace wd {

// M^dag M (eo = 0) or Mhat^dag Mhat (eo = 1) of `in` into `out` (canonical
// FP64, device) through the packed buffers A, T, B (FP64, two parity
// subfields each), with dcf = {-kappa, -kappa^2} and act = {0, 1} on the
// device: the kernels of wd_mdagm and of its allocation-free variant.
wd_status mdagm_apply(wd_ctx *c, double *out, const double *in, int eo, const double *dcf, const int *act,
                      const Field &A, const Field &T, const Field &B)
{
    hipError_t e;
    Sweep sw;
    sw.sp = SP_F64; sw.lk = c->lk64; sw.nact = 1;
    if (eo) {
        // the coefficient array is indexed by RHS id: use id 1 -> -kappa^2
        sw.active = act + 1;
        // fields are addressed as RHS id 1 with zero RHS stride
        Field a0 = sub_view(A, 0), t1 = sub_view(T, 1), b0 = sub_view(B, 0), c0 = sub_view(T, 0);
        a0.rs = t1.rs = b0.rs = c0.rs = 0;
        if ((e = pack_spinor(in, a0, 1, 0, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
        sw.coef = dcf;
        sw.P = 1; sw.dag = 0; sw.epi = EPI_PLAIN; sw.in = a0; sw.out = t1;
        WD_TRY(run_sweep(c, sw, nullptr));
        sw.P = 0; sw.epi = EPI_XPAY; sw.in = t1; sw.x = a0; sw.out = b0;
        WD_TRY(run_sweep(c, sw, nullptr));
        sw.P = 1; sw.dag = 1; sw.epi = EPI_PLAIN; sw.in = b0; sw.out = t1;
        WD_TRY(run_sweep(c, sw, nullptr));
        sw.P = 0; sw.epi = EPI_XPAY; sw.in = t1; sw.x = b0; sw.out = c0;
        WD_TRY(run_sweep(c, sw, nullptr));
        if ((e = unpack_spinor(c0, out, 1, 0, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    } else {
        sw.active = act;  // id 0 -> -kappa
        sw.coef = dcf;
        if ((e = pack_spinor(in, A, 1, 1, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "pack: %s", hipGetErrorString(e));
        sw.epi = EPI_XPAY;
        for (int pass = 0; pass < 2; pass++) {
            const Field &src = pass ? T : A;
            const Field &dst = pass ? B : T;
            sw.dag = pass;
            for (int P = 0; P < 2; P++) {
                sw.P = P;
                sw.in = sub_view(src, 1 - P);
                sw.x = sub_view(src, P);
                sw.out = sub_view(dst, P);
                WD_TRY(run_sweep(c, sw, nullptr));
            }
        }
        if ((e = unpack_spinor(B, out, 1, 1, c->g, c->stream)) != hipSuccess)
            return set_error(WD_ERR_HIP, "unpack: %s", hipGetErrorString(e));
    }
    return WD_OK;
}

}  // namespace wd
}  // extern "C++"

wd_status wd_mdagm(wd_ctx *c, double *out, const double *in, double kappa, int eo)
{
    if (!c || !out || !in) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    if (!std::isfinite(kappa)) return set_error(WD_ERR_ARG, "kappa not finite");
    WD_HIP(hipSetDevice(c->device));
    double cf[2] = {-kappa, -kappa * kappa};
    double *dcf;
    WD_TRY(upload_doubles(c, "mdm_coef", cf, 2, &dcf));
    int idx[2] = {0, 1};
    int *act;
    WD_TRY(upload_ints(c, "mdm_act", idx, 2, &act));
    Field A, T, B;
    WD_TRY(alloc_field(c, "mdm_a", SP_F64, 2, 1, &A));
    WD_TRY(alloc_field(c, "mdm_t", SP_F64, 2, 1, &T));
    WD_TRY(alloc_field(c, "mdm_b", SP_F64, 2, 1, &B));
    return mdagm_apply(c, out, in, eo, dcf, act, A, T, B);
}

wd_status wd_index_tables(const int32_t dims[4], int32_t *nb, int32_t *cb, uint8_t *par)
{
    long long V;
    WD_TRY(check_dims(dims, &V));
    if (!nb || !cb || !par) return set_error(WD_ERR_ARG, "NULL argument");
    const int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    for (long long s = 0; s < V; s++) {
        int x[4];
        long long r = s;
        for (int mu = 0; mu < 4; mu++) {
            x[mu] = (int)(r % L[mu]);
            r /= L[mu];
        }
        for (int mu = 0; mu < 4; mu++)
            for (int d = 0; d < 2; d++) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                y[mu] = (y[mu] + (d ? L[mu] - 1 : 1)) % L[mu];
                nb[s * 8 + 2 * mu + d] = (int32_t)(y[0] + (long long)L[0] * (y[1] + (long long)L[1] * (y[2] + (long long)L[2] * y[3])));
            }
        cb[s] = (int32_t)(s >> 1);
        par[s] = (uint8_t)((x[0] + x[1] + x[2] + x[3]) & 1);
    }
    return WD_OK;
}

wd_status wd_debug_device_tables(wd_ctx *c, int32_t *nb, int32_t *cb, uint8_t *par)
{
    if (!c || !nb || !cb || !par) return set_error(WD_ERR_ARG, "NULL argument");
    WD_HIP(hipSetDevice(c->device));
    hipError_t e = debug_tables(c->g, nb, cb, par, c->stream);
    if (e != hipSuccess) return set_error(WD_ERR_HIP, "debug tables: %s", hipGetErrorString(e));
    return WD_OK;
}

wd_status wd_timing_enable(wd_ctx *c, int on)
{
    if (!c) return set_error(WD_ERR_ARG, "NULL context");
    WD_HIP(hipStreamSynchronize(c->stream));
    c->timing = on != 0;
    c->ev_used = 0;
    c->t_bytes = 0;
    c->t_ms = 0;
    c->t_launches = 0;
    return WD_OK;
}

wd_status wd_timing_read(wd_ctx *c, double *total_ms, int64_t *launches, double *bytes)
{
    if (!c) return set_error(WD_ERR_ARG, "NULL context");
    WD_HIP(hipStreamSynchronize(c->stream));
    double ms = 0;
    for (size_t k = 0; k < c->ev_used; k++) {
        float t = 0;
        WD_HIP(hipEventElapsedTime(&t, c->events[k].first, c->events[k].second));
        ms += t;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = c->t_launches;
    if (bytes) *bytes = c->t_bytes;
    c->ev_used = 0;
    c->t_bytes = 0;
    c->t_launches = 0;
    return WD_OK;
}

wd_status wd_timing_report(wd_ctx *c, char *buf, size_t len)
{
    if (!c || !buf || len == 0) return set_error(WD_ERR_ARG, "NULL argument");
    WD_HIP(hipStreamSynchronize(c->stream));
    std::map<std::string, std::tuple<long long, double, double, double>> agg;
    for (size_t k = 0; k < c->ev_used; k++) {
        float t = 0;
        WD_HIP(hipEventElapsedTime(&t, c->events[k].first, c->events[k].second));
        auto &a = agg[std::get<0>(c->ev_info[k])];
        std::get<0>(a) += 1;
        std::get<1>(a) += t;
        std::get<2>(a) += std::get<1>(c->ev_info[k]);
        std::get<3>(a) += std::get<2>(c->ev_info[k]);
    }
    std::string out;
    for (auto &kv : agg) {
        char line[256];
        snprintf(line, sizeof(line), "%s;%lld;%.6f;%.1f;%.1f\n", kv.first.c_str(),
                 std::get<0>(kv.second), std::get<1>(kv.second), std::get<2>(kv.second),
                 std::get<3>(kv.second));
        out += line;
    }
    if (out.size() + 1 > len) return set_error(WD_ERR_ARG, "report needs %zu bytes", out.size() + 1);
    memcpy(buf, out.c_str(), out.size() + 1);
    return WD_OK;
}

size_t wd_bytes_required(const int32_t dims[4], int nrhs, const wd_solver_params *p)
{
    long long V;
    if (check_dims(dims, &V) != WD_OK || nrhs < 0) return 0;
    wd_solver_params d;
    wd_solver_defaults(&d);
    if (!p) p = &d;
    // fields are allocated with the padded per-parity stride
    const size_t Vh = (size_t)padded_stride((int)(V / 2));
    size_t links = (144 + 48 + 24 + 72) * 4 * (size_t)V;
    const int sp = p->prec_sloppy & 0xf;
    const size_t nsub = p->eo ? 1 : 2;
    // FP64: b, x, r, p, Ap, a full-size temporary and a one-parity temporary;
    // a mixed even-odd solve also holds the ring of sloppy search directions
    // (an FP64 solve advances its solution every iteration)
    const size_t ring = (p->eo && sp != WD_F64) ? (size_t)(kMaxRing - 1) : 0;
    size_t f64 = (6 * nsub + 1) * 192 * Vh;
    size_t sl = 0;
    if (sp != WD_F64)
        sl = (4 + ring) * spinor_site_bytes(sp == WD_F32 ? SP_F32 : SP_F16) * Vh * nsub + 96 * Vh * nsub;
    return links + (size_t)nrhs * (f64 + sl) + (size_t)nrhs * (4096 + 8 * kMaxRing);
}

}  // extern "C"
