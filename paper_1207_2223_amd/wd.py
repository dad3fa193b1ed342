"""Thin ctypes binding of libwd.so (the C-ABI declared in include/wd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions keep the C names (wd_create, wd_dslash, wd_cg_solve, ...)
and take torch CUDA tensors where the C-ABI takes device pointers.  If the
library has not been built, loading fails loudly; there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwd.so")

WD_OK, WD_ERR_ARG, WD_ERR_DIMS, WD_ERR_OOM, WD_ERR_HIP, WD_ERR_NOCONV, WD_ERR_NAN, WD_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
WD_F64, WD_F32, WD_F16, WD_I16 = 0, 1, 2, 3
WD_LINKS_F16 = 0x10
WD_LINKS_R18 = 0x20
WD_LINKS_R8 = 0x40
WD_FULL, WD_EVEN, WD_ODD = 0, 1, 2
WD_RECON_18, WD_RECON_12 = 0, 1

STATUS_NAMES = {0: "WD_OK", -1: "WD_ERR_ARG", -2: "WD_ERR_DIMS", -3: "WD_ERR_OOM", -4: "WD_ERR_HIP",
                -5: "WD_ERR_NOCONV", -6: "WD_ERR_NAN", -7: "WD_ERR_STATE"}


class WDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class wd_solver_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("prec_sloppy", C.c_int),
                ("eo", C.c_int), ("delta", C.c_double), ("poll", C.c_int), ("tuned", C.c_int),
                ("graphs", C.c_int), ("initial_guess", C.c_int)]


class wd_solver_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("true_resid", C.c_double),
                ("seconds", C.c_double), ("status", C.c_int), ("iters_fp64", C.c_int)]


class wd_hmc_params(C.Structure):
    _fields_ = [("beta", C.c_double), ("kappa", C.c_double), ("tau", C.c_double),
                ("nsteps", C.c_int), ("traj", C.c_uint32), ("seed", C.c_uint64),
                ("force_solver", wd_solver_params), ("h_solver", wd_solver_params),
                ("metropolis", C.c_int), ("chrono", C.c_int)]


class wd_hmc_result(C.Structure):
    _fields_ = [("dH", C.c_double), ("exp_mdH", C.c_double), ("plaquette", C.c_double),
                ("H_old", C.c_double), ("H_new", C.c_double), ("u", C.c_double),
                ("seconds", C.c_double), ("accepted", C.c_int), ("cg_iters", C.c_int),
                ("status", C.c_int)]


_P = C.c_void_p
_I32x4 = C.c_int32 * 4
_SIGS = {
    "wd_solver_defaults": (None, [C.POINTER(wd_solver_params)]),
    "wd_create": (C.c_int, [C.POINTER(_P), _I32x4, C.c_int, _P]),
    "wd_destroy": (C.c_int, [_P]),
    "wd_set_stream": (C.c_int, [_P, _P]),
    "wd_gauge_load": (C.c_int, [_P, _P, C.c_uint32]),
    "wd_dslash": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int]),
    "wd_dslash_shaped": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32)]),
    "wd_mdagm": (C.c_int, [_P, _P, _P, C.c_double, C.c_int]),
    "wd_mdagm_noalloc": (C.c_int, [_P, _P, _P, C.c_double, C.c_int]),
    "wd_cg_solve": (C.c_int, [_P, _P, _P, C.c_int, C.POINTER(C.c_double),
                              C.POINTER(wd_solver_params), C.POINTER(wd_solver_stats)]),
    "wd_index_tables": (C.c_int, [_I32x4, _P, _P, _P]),
    "wd_debug_device_tables": (C.c_int, [_P, _P, _P, _P]),
    "wd_bytes_required": (C.c_size_t, [_I32x4, C.c_int, C.POINTER(wd_solver_params)]),
    "wd_timing_enable": (C.c_int, [_P, C.c_int]),
    "wd_timing_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_double)]),
    "wd_timing_report": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "wd_tune": (C.c_int, [_P, C.c_int, C.c_int, C.c_char_p, C.c_size_t]),
    "wd_bench_dslash": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "wd_faces_apply": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int]),
    "wd_bench_faces": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "wd_session_create": (C.c_int, [_P, C.c_int, C.POINTER(wd_solver_params), C.POINTER(_P)]),
    "wd_session_destroy": (C.c_int, [_P]),
    "wd_session_add": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "wd_session_step": (C.c_int, [_P, C.c_int]),
    "wd_session_resize": (C.c_int, [_P, C.c_int]),
    "wd_session_capacity": (C.c_int, [_P]),
    "wd_session_poll": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(wd_solver_stats)]),
    "wd_session_take": (C.c_int, [_P, C.c_int, _P]),
    "wd_session_bytes": (C.c_size_t, [_I32x4, C.c_int, C.POINTER(wd_solver_params)]),
    "wd_hmc_defaults": (None, [C.POINTER(wd_hmc_params)]),
    "wd_hmc_draw": (C.c_int, [_P, _P, _P, C.c_uint64, C.c_uint32]),
    "wd_md_force": (C.c_int, [_P, _P, _P, _P, C.c_double, C.c_double, C.POINTER(wd_solver_params),
                              C.POINTER(C.c_int)]),
    "hmc_trajectory": (C.c_int, [_P, _P, C.POINTER(wd_hmc_params), C.POINTER(wd_hmc_result)]),
    "wd_plaquette": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "wd_polyakov": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "wd_point_propagator": (C.c_int, [_P, _P, _I32x4, C.c_double, C.POINTER(wd_solver_params),
                                      C.POINTER(wd_solver_stats)]),
    "wd_pion_correlator": (C.c_int, [_P, C.POINTER(C.c_double), _P, _I32x4]),
    "wd_last_error": (C.c_char_p, []),
    "wd_version": (C.c_char_p, []),
}

_LIB = None


def lib():
    """Load libwd.so (built by paper_1207_2223_amd/build.py); raise if absent."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading it
        # first makes libwd bind to that same runtime, so device pointers and
        # streams from torch are valid inside the library: one runtime per
        # process.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1207_2223_amd/build.py "
                              "(no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(status):
    if status != WD_OK:
        raise WDError(status, lib().wd_last_error().decode())
    return status


def _dims(dims):
    return _I32x4(*[int(v) for v in dims])


def _ptr(t, info=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (on the context's device when
    info is given)."""
    if t is None:
        return None
    if info is not None:
        _on_device(t, info, name)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _c128(t, shape_tail, name):
    import torch
    if t.dtype != torch.complex128:
        raise ValueError(f"{name} must be complex128")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [..., {shape_tail}]")
    return t


# Lattice and device of every live context and session, recorded at creation:
# the library takes raw device pointers, so a tensor with too few sites, or on
# another device, must be refused here before its pointer reaches a kernel.
class _CtxInfo:
    def __init__(self, dims, device):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.device = int(device)


_CTX = {}   # context handle value -> _CtxInfo
_SESS = {}  # session handle value -> (_CtxInfo, eo)


def _key(h):
    return h.value if isinstance(h, C.c_void_p) else int(h)


def _ctx_info(ctx):
    info = _CTX.get(_key(ctx))
    if info is None:
        raise ValueError("unknown context handle (not from wd_create, or destroyed)")
    return info


def _sites(info, parity_or_eo, full_code):
    """Sites of a field: V when parity_or_eo == full_code, else Vh."""
    return info.V if parity_or_eo == full_code else info.Vh


def _field(t, info, sites, tail, name, nrhs=None):
    """complex128 tensor holding exactly (nrhs x) sites x tail (the device is
    checked when its pointer is taken, after every size check)."""
    _c128(t, tail, name)
    per = sites * int(np.prod(tail))
    want = per if nrhs is None else int(nrhs) * per
    if t.numel() != want:
        lead = f"{nrhs} x " if nrhs is not None else ""
        raise ValueError(f"{name} has shape {tuple(t.shape)} ({t.numel()} elements), expected "
                         f"{lead}{sites} sites x {tuple(tail)} ({want} elements)")
    return t


def _on_device(t, info, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    idx = t.device.index if t.device.index is not None else 0
    if idx != info.device:
        raise ValueError(f"{name} is on device {idx}, the context on device {info.device}")


# ---------------------------------------------------------------------------
# C-ABI calls under their C names
# ---------------------------------------------------------------------------

def wd_solver_defaults():
    p = wd_solver_params()
    lib().wd_solver_defaults(C.byref(p))
    return p


def wd_create(dims, device=0, stream=None):
    h = C.c_void_p()
    _check(lib().wd_create(C.byref(h), _dims(dims), int(device), _stream_handle(stream)))
    _CTX[_key(h)] = _CtxInfo(dims, device)
    return h


def wd_destroy(ctx):
    _check(lib().wd_destroy(ctx))
    _CTX.pop(_key(ctx), None)


def wd_set_stream(ctx, stream=None):
    _check(lib().wd_set_stream(ctx, _stream_handle(stream)))


def wd_gauge_load(ctx, U, flags=WD_RECON_18):
    info = _ctx_info(ctx)
    _field(U, info, info.V, (4, 3, 3), "U")
    _check(lib().wd_gauge_load(ctx, _ptr(U, info, "U"), int(flags)))


def wd_dslash(ctx, out, inp, out_parity, dagger=0, prec=WD_F64):
    info = _ctx_info(ctx)
    n = _sites(info, int(out_parity), WD_FULL)
    _field(out, info, n, (4, 3), "out")
    _field(inp, info, n, (4, 3), "in")
    _check(lib().wd_dslash(ctx, _ptr(out, info, "out"), _ptr(inp, info, "in"), int(out_parity),
                           int(dagger), int(prec)))


def wd_dslash_shaped(ctx, out, inp, out_parity, dagger=0, prec=WD_F64, shape=None):
    """out, inp: complex128 [nrhs, Vh, 4, 3] (or [Vh, 4, 3]); shape: None or
    (block, nr, rl, tile order, work-group cap)."""
    info = _ctx_info(ctx)
    nrhs = 1 if inp.dim() == 3 else inp.shape[0]
    if tuple(out.shape) != tuple(inp.shape):
        raise ValueError(f"out has shape {tuple(out.shape)}, in {tuple(inp.shape)}: they must match")
    _field(inp, info, info.Vh, (4, 3), "in", nrhs)
    _field(out, info, info.Vh, (4, 3), "out", nrhs)
    sh = None if shape is None else (C.c_int32 * 5)(*[int(v) for v in shape])
    _check(lib().wd_dslash_shaped(ctx, _ptr(out, info, "out"), _ptr(inp, info, "in"), int(nrhs),
                                  int(out_parity), int(dagger), int(prec), sh))


def wd_mdagm(ctx, out, inp, kappa, eo=1):
    info = _ctx_info(ctx)
    n = info.Vh if eo else info.V
    _field(out, info, n, (4, 3), "out")
    _field(inp, info, n, (4, 3), "in")
    _check(lib().wd_mdagm(ctx, _ptr(out, info, "out"), _ptr(inp, info, "in"), float(kappa), int(eo)))


def wd_mdagm_noalloc(ctx, out, inp, kappa, eo=1):
    """wd_mdagm without device allocation (a fixed device scratch array)."""
    info = _ctx_info(ctx)
    n = info.Vh if eo else info.V
    _field(out, info, n, (4, 3), "out")
    _field(inp, info, n, (4, 3), "in")
    _check(lib().wd_mdagm_noalloc(ctx, _ptr(out, info, "out"), _ptr(inp, info, "in"), float(kappa), int(eo)))


def wd_cg_solve(ctx, x, phi, kappa, params=None, check=True):
    """x, phi: complex128 [nrhs, sites, 4, 3] (or [sites, 4, 3]); kappa: float
    or sequence of nrhs floats.  Returns (status, list of stats dicts)."""
    info = _ctx_info(ctx)
    p = params if params is not None else wd_solver_defaults()
    nrhs = 1 if phi.dim() == 3 else phi.shape[0]
    if tuple(x.shape) != tuple(phi.shape):
        raise ValueError(f"x has shape {tuple(x.shape)}, phi {tuple(phi.shape)}: they must match")
    n = info.Vh if p.eo else info.V
    _field(phi, info, n, (4, 3), "phi", nrhs)
    _field(x, info, n, (4, 3), "x", nrhs)
    ks = [float(kappa)] * nrhs if np.isscalar(kappa) else [float(k) for k in kappa]
    if len(ks) != nrhs:
        raise ValueError("one kappa per right-hand side")
    karr = (C.c_double * nrhs)(*ks)
    st = (wd_solver_stats * nrhs)()
    status = lib().wd_cg_solve(ctx, _ptr(x, info, "x"), _ptr(phi, info, "phi"), nrhs, karr, C.byref(p), st)
    if check and status not in (WD_OK, WD_ERR_NOCONV, WD_ERR_NAN):
        _check(status)
    stats = [dict(iters=s.iters, iters_fp64=s.iters_fp64, reliable_updates=s.reliable_updates, true_resid=s.true_resid,
                  seconds=s.seconds, status=s.status) for s in st]
    return status, stats


def wd_index_tables(dims):
    V = int(np.prod(dims))
    nb = np.zeros((V, 8), np.int32)
    cb = np.zeros(V, np.int32)
    par = np.zeros(V, np.uint8)
    _check(lib().wd_index_tables(_dims(dims), nb.ctypes.data_as(_P), cb.ctypes.data_as(_P),
                                 par.ctypes.data_as(_P)))
    return nb, cb, par


def wd_debug_device_tables(ctx, nb, cb, par):
    import torch
    info = _ctx_info(ctx)
    for name, t, n, dt in (("nb", nb, 8 * info.V, torch.int32), ("cb", cb, info.V, torch.int32),
                           ("par", par, info.V, torch.uint8)):
        if t.dtype != dt or t.numel() != n:
            raise ValueError(f"{name} must be {n} elements of {dt}, got {t.numel()} of {t.dtype}")
    _check(lib().wd_debug_device_tables(ctx, _ptr(nb, info, "nb"), _ptr(cb, info, "cb"),
                                        _ptr(par, info, "par")))


def wd_bytes_required(dims, nrhs, params=None):
    p = C.byref(params) if params is not None else None
    return int(lib().wd_bytes_required(_dims(dims), int(nrhs), p))


def wd_timing_enable(ctx, on=True):
    _check(lib().wd_timing_enable(ctx, int(bool(on))))


def wd_timing_read(ctx):
    ms = C.c_double()
    n = C.c_int64()
    b = C.c_double()
    _check(lib().wd_timing_read(ctx, C.byref(ms), C.byref(n), C.byref(b)))
    return ms.value, n.value, b.value


def wd_timing_report(ctx):
    """{kernel name: (launches, total_ms, algorithmic_bytes, output_site_rhs)} since the last
    reset."""
    buf = C.create_string_buffer(1 << 16)
    _check(lib().wd_timing_report(ctx, buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms, b, u = line.split(";")
        out[name] = (int(n), float(ms), float(b), float(u))
    return out


def wd_tune(ctx, nrhs, prec):
    """Autotune the solver's stencil sweeps; returns the report lines as dicts."""
    buf = C.create_string_buffer(1 << 14)
    _check(lib().wd_tune(ctx, int(nrhs), int(prec), buf, len(buf)))
    rows = []
    for line in buf.value.decode().splitlines():
        f = line.split(";")
        d = {"sweep": f[0]}
        for kv in f[1:]:
            k, v = kv.split("=")
            try:
                d[k] = float(v) if "." in v else int(v)
            except ValueError:
                d[k] = v
        rows.append(d)
    return rows


def wd_bench_dslash(ctx, nrhs, prec, epi=0, iters=20, tuned=1):
    """(ms per sweep, algorithmic bytes per sweep) of the stencil micro-benchmark."""
    ms = C.c_double()
    by = C.c_double()
    _check(lib().wd_bench_dslash(ctx, int(nrhs), int(prec), int(epi), int(iters), int(tuned),
                                 C.byref(ms), C.byref(by)))
    return ms.value, by.value


def wd_faces_apply(ctx, out, inp, out_parity, dagger=0, prec=WD_F64):
    """Face terms across a cut along t of one hopping sweep (include/wd.h)."""
    info = _ctx_info(ctx)
    _field(out, info, info.Vh, (4, 3), "out")
    _field(inp, info, info.Vh, (4, 3), "in")
    _check(lib().wd_faces_apply(ctx, _ptr(out, info, "out"), _ptr(inp, info, "in"), int(out_parity),
                                int(dagger), int(prec)))


def wd_bench_faces(ctx, prec, iters=20):
    """(pack ms, update ms, pack bytes, update bytes) of the face kernels."""
    v = [C.c_double() for _ in range(4)]
    _check(lib().wd_bench_faces(ctx, int(prec), int(iters), *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def wd_session_create(ctx, max_rhs, params=None):
    info = _ctx_info(ctx)
    h = C.c_void_p()
    p = params if params is not None else wd_solver_defaults()
    _check(lib().wd_session_create(ctx, int(max_rhs), C.byref(p), C.byref(h)))
    _SESS[_key(h)] = (info, int(p.eo))
    return h


def wd_session_destroy(sess):
    _check(lib().wd_session_destroy(sess))
    _SESS.pop(_key(sess), None)


def _sess_info(sess):
    s = _SESS.get(_key(sess))
    if s is None:
        raise ValueError("unknown session handle (not from wd_session_create, or destroyed)")
    info, eo = s
    return info, (info.Vh if eo else info.V)


def wd_session_add(sess, phi, kappa):
    """phi: complex128 [nrhs, sites, 4, 3] device tensor; returns the slots."""
    info, n = _sess_info(sess)
    nrhs = 1 if phi.dim() == 3 else phi.shape[0]
    _field(phi, info, n, (4, 3), "phi", nrhs)
    ks = [float(kappa)] * nrhs if np.isscalar(kappa) else [float(k) for k in kappa]
    if len(ks) != nrhs:
        raise ValueError("one kappa per right-hand side")
    slots = (C.c_int32 * nrhs)()
    _check(lib().wd_session_add(sess, _ptr(phi, info, "phi"), nrhs, (C.c_double * nrhs)(*ks), slots))
    return list(slots)


def wd_session_step(sess, k_iters):
    _check(lib().wd_session_step(sess, int(k_iters)))


def wd_session_resize(sess, max_rhs):
    _check(lib().wd_session_resize(sess, int(max_rhs)))


def wd_session_capacity(sess):
    return int(lib().wd_session_capacity(sess))


def wd_session_poll(sess, max_rhs=None):
    """(states list, stats list) for every slot."""
    cap = wd_session_capacity(sess)
    if max_rhs is not None and max_rhs != cap:
        raise ValueError(f"the session has {cap} slots, not {max_rhs}")
    max_rhs = cap
    state = (C.c_int32 * max_rhs)()
    st = (wd_solver_stats * max_rhs)()
    _check(lib().wd_session_poll(sess, state, st))
    stats = [dict(iters=s.iters, iters_fp64=s.iters_fp64, reliable_updates=s.reliable_updates, true_resid=s.true_resid,
                  seconds=s.seconds, status=s.status) for s in st]
    return list(state), stats


def wd_session_take(sess, slot, x):
    info, n = _sess_info(sess)
    _field(x, info, n, (4, 3), "x")
    _check(lib().wd_session_take(sess, int(slot), _ptr(x, info, "x")))


def wd_session_bytes(dims, max_rhs, params=None):
    p = C.byref(params) if params is not None else None
    return int(lib().wd_session_bytes(_dims(dims), int(max_rhs), p))


def wd_hmc_defaults():
    h = wd_hmc_params()
    lib().wd_hmc_defaults(C.byref(h))
    return h


def wd_hmc_draw(ctx, P, chi, seed, traj):
    info = _ctx_info(ctx)
    _field(P, info, info.V, (4, 3, 3), "P")
    _field(chi, info, info.Vh, (4, 3), "chi")
    _check(lib().wd_hmc_draw(ctx, _ptr(P, info, "P"), _ptr(chi, info, "chi"), int(seed), int(traj)))


def wd_md_force(ctx, F, U, phi, kappa, beta, params=None):
    """F = F_g + F_f (even-odd action); returns the solve's iteration count."""
    info = _ctx_info(ctx)
    _field(F, info, info.V, (4, 3, 3), "F")
    _field(U, info, info.V, (4, 3, 3), "U")
    _field(phi, info, info.Vh, (4, 3), "phi")
    it = C.c_int(0)
    p = params if params is not None else wd_solver_defaults()
    _check(lib().wd_md_force(ctx, _ptr(F, info, "F"), _ptr(U, info, "U"), _ptr(phi, info, "phi"),
                             float(kappa), float(beta),
                             C.byref(p), C.byref(it)))
    return it.value


def hmc_trajectory(ctx, U, params, check=True):
    """One trajectory; U is updated in place when accepted.  Returns a dict."""
    info = _ctx_info(ctx)
    _field(U, info, info.V, (4, 3, 3), "U")
    r = wd_hmc_result()
    st = lib().hmc_trajectory(ctx, _ptr(U, info, "U"), C.byref(params), C.byref(r))
    if check and st not in (WD_OK, WD_ERR_NOCONV, WD_ERR_NAN):
        _check(st)
    return {k: getattr(r, k) for k, _ in wd_hmc_result._fields_}


def hmc_params(beta=5.6, kappa=0.156, tau=1.0, nsteps=50, seed=1, traj=0, force=None, h=None,
               metropolis=True, chrono=False):
    p = wd_hmc_defaults()
    p.beta, p.kappa, p.tau, p.nsteps, p.seed, p.traj = (float(beta), float(kappa), float(tau),
                                                        int(nsteps), int(seed), int(traj))
    p.metropolis = 1 if metropolis else 0
    p.chrono = int(chrono)
    if force is not None:
        p.force_solver = force
    if h is not None:
        p.h_solver = h
    return p


def wd_plaquette(ctx, U):
    info = _ctx_info(ctx)
    _field(U, info, info.V, (4, 3, 3), "U")
    out = C.c_double(0)
    _check(lib().wd_plaquette(ctx, _ptr(U, info, "U"), C.byref(out)))
    return out.value


def wd_polyakov(ctx, U):
    """Complex Polyakov loop of U ([V][4][3][3] complex128 device tensor)."""
    info = _ctx_info(ctx)
    _field(U, info, info.V, (4, 3, 3), "U")
    out = (C.c_double * 2)()
    _check(lib().wd_polyakov(ctx, _ptr(U, info, "U"), out))
    return complex(out[0], out[1])


def wd_point_propagator(ctx, psi, src, kappa, params=None, check=True):
    """psi: complex128 [12, V, 4, 3] device tensor (written); returns
    (status, stats list)."""
    info = _ctx_info(ctx)
    if psi.dim() != 4 or psi.shape[0] != 12:
        raise ValueError("psi must be [12, V, 4, 3]")
    _field(psi, info, info.V, (4, 3), "psi", 12)
    p = params if params is not None else wd_solver_defaults()
    st = (wd_solver_stats * 12)()
    status = lib().wd_point_propagator(ctx, _ptr(psi, info, "psi"), _dims(src), float(kappa),
                                       C.byref(p), st)
    if check and status not in (WD_OK, WD_ERR_NOCONV, WD_ERR_NAN):
        _check(status)
    stats = [dict(iters=s.iters, iters_fp64=s.iters_fp64, reliable_updates=s.reliable_updates,
                  true_resid=s.true_resid, seconds=s.seconds, status=s.status) for s in st]
    return status, stats


def wd_pion_correlator(ctx, psi, src, Lt):
    info = _ctx_info(ctx)
    if psi.dim() != 4 or psi.shape[0] != 12:
        raise ValueError("psi must be [12, V, 4, 3]")
    _field(psi, info, info.V, (4, 3), "psi", 12)
    corr = (C.c_double * int(Lt))()
    _check(lib().wd_pion_correlator(ctx, corr, _ptr(psi, info, "psi"), _dims(src)))
    return np.array(corr[:])


def wd_last_error():
    return lib().wd_last_error().decode()


def wd_version():
    return lib().wd_version().decode()


def solver_params(tol=1e-10, maxiter=20000, prec=WD_F64, eo=1, delta=0.1, poll=8, tuned=0, graphs=1,
                  initial_guess=0):
    p = wd_solver_defaults()
    p.tol, p.maxiter, p.prec_sloppy, p.eo, p.delta, p.poll, p.tuned, p.graphs = (
        float(tol), int(maxiter), int(prec), int(eo), float(delta), int(poll), int(tuned), int(graphs))
    p.initial_guess = int(initial_guess)
    return p


class Lattice:
    """A context for one lattice (owns the packed gauge field)."""

    def __init__(self, dims, device=0, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.device = device
        self.ctx = wd_create(self.dims, device, stream)

    def close(self):
        if self.ctx is not None:
            wd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gauge_load(self, U, recon=18):
        wd_gauge_load(self.ctx, U, WD_RECON_12 if recon == 12 else WD_RECON_18)

    def dslash(self, out, inp, out_parity, dagger=0, prec=WD_F64):
        wd_dslash(self.ctx, out, inp, out_parity, dagger, prec)

    def mdagm(self, out, inp, kappa, eo=1):
        wd_mdagm(self.ctx, out, inp, kappa, eo)

    def faces_apply(self, out, inp, out_parity, dagger=0, prec=WD_F64):
        for name, t in (("out", out), ("in", inp)):
            if tuple(t.shape) != (self.V // 2, 4, 3):
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected ({self.V // 2}, 4, 3)")
        wd_faces_apply(self.ctx, out, inp, out_parity, dagger, prec)

    def cg_solve(self, x, phi, kappa, params=None, check=True):
        return wd_cg_solve(self.ctx, x, phi, kappa, params, check)

    def plaquette(self, U):
        if tuple(U.shape) != (self.V, 4, 3, 3):
            raise ValueError(f"U has shape {tuple(U.shape)}, expected ({self.V}, 4, 3, 3)")
        return wd_plaquette(self.ctx, U)

    def polyakov(self, U):
        if tuple(U.shape) != (self.V, 4, 3, 3):
            raise ValueError(f"U has shape {tuple(U.shape)}, expected ({self.V}, 4, 3, 3)")
        return wd_polyakov(self.ctx, U)

    def point_propagator(self, psi, src, kappa, params=None, check=True):
        if tuple(psi.shape) != (12, self.V, 4, 3):
            raise ValueError(f"psi has shape {tuple(psi.shape)}, expected (12, {self.V}, 4, 3)")
        return wd_point_propagator(self.ctx, psi, src, kappa, params, check)

    def pion_correlator(self, psi, src):
        if tuple(psi.shape) != (12, self.V, 4, 3):
            raise ValueError(f"psi has shape {tuple(psi.shape)}, expected (12, {self.V}, 4, 3)")
        return wd_pion_correlator(self.ctx, psi, src, self.dims[3])
