// wd_internal.h -- host-side internals shared by the library's translation
// units: the context, field descriptors, kernel argument blocks, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/wd.h"
#include "wd_device.h"

namespace wd {

wd_status set_error(wd_status st, const char *fmt, ...);

#define WD_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::wd::set_error(WD_ERR_HIP, "%s failed: %s (%s:%d)", #call,                   \
                                   hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

#define WD_TRY(expr)                                                                              \
    do {                                                                                          \
        wd_status s_ = (expr);                                                                    \
        if (s_ != WD_OK) return s_;                                                               \
    } while (0)

enum { EPI_PLAIN = 0, EPI_XPAY = 1, EPI_CGUPD = 2 };

// A batch of spinor fields of one precision: RHS id r, parity subfield s
// starts at base + r*rs + s*ss.  nsub = 1 (one parity) or 2 (full lattice).
struct Field {
    char *base = nullptr;
    long long rs = 0;
    long long ss = 0;
    int sp = SP_F64;
    int nsub = 1;
    int cs = 0;  // chunk stride (sites) of the structure-of-arrays layout
    char *sub(int rid, int s) const { return base + rid * rs + s * ss; }
};

// Stencil kernel arguments (passed by value).
struct DslashArgs {
    Geom g;
    int P;                 // output parity
    const char *links;
    const char *in;        // input subfield of RHS 0 (parity 1-P)
    long long in_rs;
    char *out;             // output subfield of RHS 0 (parity P)
    long long out_rs;
    const char *x;         // xpay: out = x + coef*D in
    long long x_rs;
    const double *coef;    // [rid]
    char *r;               // CG update: r -= alpha (x + coef*D in)
    long long r_rs;
    const double *alpha;   // [rid]
    const int *active;     // RHS ids processed by this launch
    int nact;
    int G;                 // RHS groups of RL*NR per tile
    int remap;             // tile order: 0 dispatch order, 1 XCD-contiguous, 2 XCD z-slabs
    int tpp;               // remap >= 2: tiles per (z, t) plane
    int nzl;               // remap 2-4: z planes per XCD; 5-6: t planes per XCD
    int nys;               // remap >= 2: stripes per plane (1, 2, 4 for remap 2, 3, 4)
    int tch;               // t-walking orders: t planes per work-group
    double *partial;       // partial[rid*pstride + pw_off + site/16] = sum |out|^2 (or |r|^2)
    int pstride;
    int pw_off;
    unsigned lds;          // dynamic LDS bytes per work-group (unused by the kernel: caps occupancy)
    // CG alpha finalized by the first fin_blocks work-groups (one per active
    // RHS, before the stencil's tiles): alpha = rr / sum of fin_partial
    // (fin_nw partials per RHS, stride fin_pstride), written to fin_alpha
    // and fin_out (if not null); 0 = none
    int fin_blocks;
    int fin_nw;
    int fin_pstride;
    const double *fin_partial;
    double *fin_rr;
    double *fin_alpha;
    double *fin_out;
};

// Launch shape of one stencil sweep: threads per work-group, RHS per lane
// (nr), lanes per site (rl), tile order (remap: 0 dispatch order,
// 1 contiguous tile range per XCD, 2 z-slab per XCD walked z-fastest, ...),
// and an optional cap on work-groups per CU (occ).
struct TuneCfg {
    int block = 128;
    int nr = 1;
    int rl = 1;
    int remap = 1;
    int occ = 0;  // 0, or at most occ work-groups per CU (enforced through dynamic LDS)
    int lnt = 0;  // 1: links loaded non-temporally (FP32 12/8-real, FP64 12-real; register-tiled, rl 1, nr 1-2)
};
// Whether a shape of a sweep with links lk may take lnt = 1, and the
// non-temporal launch variant of a link format (-1: none).
bool lnt_ok(int sp, int lk, const TuneCfg &t);
inline int lnt_variant(int lk)
{
    return lk == LK_F32_12 ? LK_F32_12N : (lk == LK_F64_12 ? LK_F64_12N : (lk == LK_F32_8 ? LK_F32_8N : -1));
}

// LDS per CU on gfx950, and the dynamic LDS per work-group that lets at most
// occ work-groups share a CU (occ in 2..kMaxOcc; 0 = no cap).
constexpr unsigned kLdsPerCU = 160u * 1024u;
constexpr int kMaxOcc = 8;
inline unsigned occ_lds_bytes(int occ) { return occ > 0 ? kLdsPerCU / (unsigned)(occ + 1) + 1024u : 0u; }

hipError_t dslash_launch(const DslashArgs &a, int sp, int lk, int nr, int rl, int dag, int epi,
                         int block, int grid, hipStream_t s);
bool dslash_shape_supported(int sp, int lk, int nr, int rl);
// The LDS-staged t-walking stencil (tile orders kLdsOrder0 and up: work-groups
// of 256 threads walking kLdsChunk[order - kLdsOrder0] t-planes of one
// z-plane column, NR RHS per lane, one lane per site).
hipError_t dslash_lds_launch(const DslashArgs &a, int sp, int lk, int nr, int dag, int epi, int grid,
                             unsigned lds_bytes, hipStream_t s);
bool dslash_lds_supported(int sp, int lk, int nr);
// The t-walking stencil with the t neighbours in registers (tile orders
// kTwOrder0 and up: work-groups of `block` threads, one lane per site of a
// block-site tile of one (z, t) plane, walking tw_chunk(order) t-planes).
hipError_t dslash_tw_launch(const DslashArgs &a, int sp, int lk, int nr, int dag, int epi, int block, int grid,
                            hipStream_t s);
bool dslash_tw_supported(int sp, int lk, int nr);

// BLAS-1 / reductions (blas.hip).  All take an active-RHS list.
enum { FIN_STORE = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RR = 3 };
hipError_t blas_norm(const Field &a, int Vh, const int *active, int nact, double *partial,
                     int pstride, hipStream_t s);
hipError_t blas_p_update(const Field &p, const Field &r, const double *beta, int Vh,
                         const int *active, int nact, hipStream_t s);
// The CG search-direction update of an even-odd iteration with the solution
// update deferred: p_dst = r + beta p[m-1] with p[j] the directions of the
// last m iterations (slots of a ring, p[m-1] the current one); with flush,
// first x += alpha_j p[j] for j = 0 .. m-1 in that order (alpha_j =
// ahist[j*ahs + rid]), the same roundings as advancing x every iteration.
constexpr int kMaxRing = 8;
hipError_t blas_p_update_ring(const Field *p, int m, const Field &pdst, const Field &r, const double *beta,
                              bool flush, const Field &x, const double *ahist, int ahs, int Vh,
                              const int *active, int nact, hipStream_t s);
hipError_t blas_cg_update(const Field &x, const Field &p, const Field &r, const Field &Ap,
                          const double *alpha, int Vh, const int *active, int nact,
                          double *partial, int pstride, hipStream_t s);
hipError_t blas_copy(const Field &dst, const Field &src, int Vh, const int *active, int nact,
                     hipStream_t s);
hipError_t blas_add_zero(const Field &xhi, const Field &xs, int Vh, const int *active, int nact,
                         hipStream_t s);
hipError_t blas_resid(const Field &r, const Field &b, const Field &Ap, int Vh, const int *active,
                      int nact, double *partial, int pstride, hipStream_t s);
hipError_t blas_zero(const Field &a, int Vh, const int *active, int nact, hipStream_t s);
hipError_t blas_cdot(const Field &a, const Field &b, int Vh, const int *active, int nact,
                     double *pre, double *pim, int pstride, hipStream_t s);
hipError_t blas_orth(const Field &p, const Field &r, const double *dre, const double *dim,
                     const double *rr, int Vh, const int *active, int nact, hipStream_t s);
hipError_t blas_axpy_const(const Field &p, const Field &r, double a, int Vh, const int *active,
                           int nact, hipStream_t s);
hipError_t blas_xpay_ratio(const Field &p, const Field &r, const double *num, const double *den, int Vh,
                           const int *active, int nact, hipStream_t s);
hipError_t blas_finalize(const double *partial, int pstride, int nw, const int *active, int nact,
                         int mode, double *rr, double *alpha, double *beta, double *out,
                         hipStream_t s);
// Reductions are formed from partial sums over groups of 16 consecutive sites.
inline int ngroups_of(int nsites) { return (nsites + 15) / 16; }

// Packing between the canonical complex128 layouts and the internal ones (pack.hip).
hipError_t pack_gauge(const double *U, char *dst, int lk, const Geom &g, hipStream_t s);
// mode 0: src/dst are parity fields ([Vh][4][3] cb order <-> one subfield);
// mode 1: full fields ([V][4][3] lex order <-> two subfields).
hipError_t pack_spinor(const double *src, const Field &dst, int nrhs, int mode, const Geom &g,
                       hipStream_t s);
hipError_t unpack_spinor(const Field &src, double *dst, int nrhs, int mode, const Geom &g,
                         hipStream_t s);
hipError_t debug_tables(const Geom &g, int32_t *nb, int32_t *cb, uint8_t *par, hipStream_t s);

}  // namespace wd

// The context: one lattice on one device.
struct wd_ctx {
    int device = 0;
    int lds_max = 0;  // bytes of LDS a work-group may use on this device
    hipStream_t stream = nullptr;
    int dims[4] = {0, 0, 0, 0};
    long long V = 0, Vh = 0;
    wd::Geom g{};

    bool have_gauge = false;
    int sessions = 0;  // solver sessions open on this context
    int lk64 = wd::LK_F64_18;
    char *links64 = nullptr;
    char *links32 = nullptr;
    char *links16 = nullptr;
    char *links32r = nullptr;  // FP32 18-real
    char *links8 = nullptr;    // FP32 8-real

    // named, growable device workspaces
    std::map<std::string, std::pair<void *, size_t>> ws;
    void *pinned[2] = {nullptr, nullptr};   // [0] uploads, [1] downloads
    size_t pinned_bytes[2] = {0, 0};

    // stencil timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    std::vector<std::tuple<std::string, double, double>> ev_info;  // name, bytes, site-RHS
    size_t ev_used = 0;
    double t_bytes = 0;
    double t_ms = 0;
    long long t_launches = 0;

    // launch shapes chosen by the autotuner, keyed by sweep description, and
    // whether the current call uses them
    std::map<std::string, wd::TuneCfg> tuned;
    bool use_tuned = false;
    unsigned tune_gen = 0;  // bumped whenever `tuned` changes

    // CG steps captured as HIP graphs (solver.hip), keyed by everything their
    // kernel arguments depend on; a bounded FIFO.  Captured on a private
    // stream, replayed on `stream`.
    std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
    hipStream_t capture_stream = nullptr;
};

namespace wd {

wd_status ws_get(wd_ctx *c, const std::string &name, size_t bytes, void **ptr);
wd_status pinned_get(wd_ctx *c, int slot, size_t bytes, void **ptr);
wd_status alloc_field(wd_ctx *c, const std::string &name, int sp, int nsub, int nrhs, Field *f);
const char *link_ptr(const wd_ctx *c, int lk);
// Storage of an operator precision code (wd_prec | WD_LINKS_F16 | WD_LINKS_R18):
// spinor format, link format and solution-accumulator format.
wd_status decode_prec(const wd_ctx *c, int prec, int *sp, int *lk, int *xp);

// One stencil sweep over the active RHS (dispatch + optional timing).
struct Sweep {
    int sp = SP_F64;
    int lk = LK_F64_18;
    int dag = 0;
    int epi = EPI_PLAIN;
    int P = 0;
    const char *links = nullptr;  // another copy of the packed links (else the context's)
    Field in, out, x, r;
    const double *coef = nullptr;
    const double *alpha = nullptr;
    const int *active = nullptr;
    int nact = 0;
    double *partial = nullptr;
    int pstride = 0;
    int pw_off = 0;
    // optional: the CG alpha of the partials fin_partial, finalized inside
    // this sweep by extra work-groups (see DslashArgs)
    const double *fin_partial = nullptr;
    int fin_nw = 0;
    int fin_pstride = 0;
    double *fin_rr = nullptr;
    double *fin_alpha = nullptr;
    double *fin_out = nullptr;
};
wd_status run_sweep(wd_ctx *c, const Sweep &sw, const TuneCfg *cfg);
wd_status upload_doubles(wd_ctx *c, const std::string &name, const double *v, int n, double **dev);
wd_status upload_ints(wd_ctx *c, const std::string &name, const int *v, int n, int **dev);
Field sub_view(const Field &f, int s);
TuneCfg default_cfg(int sp);
// Whether the z-slab tile order (remap 2) applies to tiles of spb sites.
// Tile orders: 0 plain, 1 XCD round-robin, 2-4 z-slab per XCD in 1/2/4
// y-stripes, 5-6 t-slab per XCD walked t-fastest, 7 z-slab per XCD with the
// RHS groups outermost.
constexpr int kTileOrders = 8;
bool slab_order_ok(const Geom &g, int spb, int remap = 2);
// Tile orders kLdsOrder0 .. kLdsOrder0 + kLdsOrders - 1: the LDS-staged
// t-walking kernel with lds_chunk(order) t-planes per work-group (256
// threads, one lane per site, no work-group cap).  It applies when a plane of
// one parity has a multiple of 64 sites and at most 512, Lz is a multiple of
// 8, Lt of the chunk, and three input planes of the RHS group fit in LDS.
constexpr int kLdsOrder0 = kTileOrders;
constexpr int kLdsOrders = 3;
inline int lds_chunk(int remap) { return 4 << (remap - kLdsOrder0); }
inline bool is_lds_order(int remap) { return remap >= kLdsOrder0 && remap < kLdsOrder0 + kLdsOrders; }
bool lds_order_ok(const wd_ctx *c, int sp, int lk, int nr, int remap);
unsigned lds_order_bytes(const wd_ctx *c, int sp, int nr);
// Tile orders kTwOrder0 .. kTwOrder0 + kTwOrders - 1: the t-walking kernel
// with the t neighbours held in registers, tw_chunk(order) t-planes per
// work-group.  It applies to FP16 spinors when a plane of one parity holds a
// whole number of block-site tiles, Lz is a multiple of 8 and Lt of the
// chunk; one lane per site (rl = 1); a cap on work-groups per CU is allowed.
constexpr int kTwOrder0 = kLdsOrder0 + kLdsOrders;
constexpr int kTwOrders = 3;
inline int tw_chunk(int remap) { return 4 << (remap - kTwOrder0); }
inline bool is_tw_order(int remap) { return remap >= kTwOrder0 && remap < kTwOrder0 + kTwOrders; }
bool tw_order_ok(const wd_ctx *c, int sp, int lk, int nr, int rl, int block, int remap);
inline int remap_stripes(int remap) { return remap <= 2 || remap >= 5 ? 1 : (remap == 3 ? 2 : 4); }
inline int remap_slab_dim(int remap) { return (remap == 5 || remap == 6) ? 3 : 2; }
const TuneCfg *tuned_cfg(const wd_ctx *c, const Sweep &sw);
double sweep_bytes(const wd_ctx *c, const Sweep &sw);
wd_status mdagm_apply(wd_ctx *c, double *out, const double *in, int eo, const double *dcf, const int *act,
                      const Field &A, const Field &T, const Field &B);
// The allocation-free entry points' device scratch array (noalloc.hip): its
// address on `device` is looked up once, with that device current (called by
// wd_create), and kept per device.
wd_status scratch_setup(int device);

}  // namespace wd
