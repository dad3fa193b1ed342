// noalloc.hip -- an allocation-free variant of wd_mdagm for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid it).
//
// The packed operand, the two temporaries of the four stencil sweeps and the
// two device scalars wd_mdagm keeps in context workspaces live here in one
// file-scope device array, `scratch`, of kScratchBytes per GPU (held by each
// GPU the library runs on until the process ends).  Its device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, when the first context on that device is created (wd_create), and
// only that address is handed to kernels.  The entry point itself calls no
// allocating routine and no host-device copy: the scalars are written by a
// one-thread kernel.  Every call on one GPU uses that GPU's array, so calls
// that overlap on one GPU (different streams or threads) race; the array
// keeps the last call's contents, and nothing in it is read before this call
// has written it.
#include <cmath>
#include <mutex>

#include "wd_internal.h"

namespace wd {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;
constexpr size_t kScalarBytes = 512;  // {-kappa, -kappa^2} and the id list {0, 1}

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

__global__ void k_noalloc_scalars(double *coef, int *ids, double c1, double c2)
{
    if (threadIdx.x == 0) {
        coef[0] = c1;
        coef[1] = c2;
        ids[0] = 0;
        ids[1] = 1;
    }
}

void *scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
}

}  // namespace

wd_status scratch_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (device < 0 || device >= kMaxDevices)
        return set_error(WD_ERR_ARG, "device %d beyond the %d the library tracks", device, kMaxDevices);
    if (g_ptr[device]) return WD_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(WD_ERR_HIP, "device scratch address on device %d: %s", device, hipGetErrorString(e));
    g_ptr[device] = p;
    return WD_OK;
}

}  // namespace wd

using namespace wd;

extern "C" wd_status wd_mdagm_noalloc(wd_ctx *c, double *out, const double *in, double kappa, int eo)
{
    if (!c || !out || !in) return set_error(WD_ERR_ARG, "NULL argument");
    if (!c->have_gauge) return set_error(WD_ERR_STATE, "no gauge field loaded");
    if (!std::isfinite(kappa)) return set_error(WD_ERR_ARG, "kappa not finite");
    char *base = (char *)scratch_ptr(c->device);
    if (!base) return set_error(WD_ERR_STATE, "no device scratch on device %d (context not from wd_create?)", c->device);
    // wd_mdagm's packed FP64 operand A and temporaries T, B: the full
    // operator uses both parity subfields of each (6 subfields), the
    // even-odd one subfield of A and B and both of T (4)
    const long long sub = ((long long)spinor_site_bytes(SP_F64) * c->g.cs + 255) / 256 * 256;
    const size_t need = kScalarBytes + (size_t)((eo ? 4 : 6) * sub);
    if (need > kScratchBytes)
        return set_error(WD_ERR_ARG,
                         "the allocation-free M^dag M needs %zu bytes of device scratch on this lattice (Vh = %lld), "
                         "more than its fixed %zu",
                         need, c->Vh, kScratchBytes);
    WD_HIP(hipSetDevice(c->device));
    double *dcf = (double *)base;
    int *act = (int *)(base + 256);
    Field f;
    f.sp = SP_F64;
    f.nsub = 2;
    f.cs = c->g.cs;
    f.ss = sub;
    f.rs = 2 * sub;
    Field A = f, T = f, B = f;
    A.base = base + kScalarBytes;
    T.base = A.base + (eo ? 1 : 2) * sub;
    B.base = T.base + 2 * sub;
    hipLaunchKernelGGL(k_noalloc_scalars, dim3(1), dim3(64), 0, c->stream, dcf, act, -kappa, -kappa * kappa);
    WD_HIP(hipGetLastError());
    // no per-launch timing events here (event creation allocates)
    const bool timing = c->timing;
    c->timing = false;
    const wd_status st = mdagm_apply(c, out, in, eo, dcf, act, A, T, B);
    c->timing = timing;
    return st;
}
