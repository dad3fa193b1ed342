"""ctypes binding of the C oracle (oracle/wdref.c) on numpy complex128 arrays.

TEST INFRASTRUCTURE ONLY.  Layouts (canonical, complex128):
  spinor  [V][4][3]   (lex order)         parity field [Vh][4][3] (cb order)
  links   [V][4][3][3]                    momenta / forces: same as links
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_PATH = None  # another build of the same source (use_library), else the in-tree one


def use_library(path):
    """Load the oracle from `path` (another build of wdref.c, e.g. one
    compiled for the host it runs on) for every later call."""
    global _LIB, _PATH
    _PATH = path
    _LIB = None
    return lib()


def lib():
    global _LIB
    if _LIB is None:
        path = _PATH or os.path.join(_HERE, "liboracle_wd.so")
        if not os.path.exists(path):
            from oracle import build
            build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i32p = C.POINTER(C.c_int32)
        d = C.c_double
        sig = {
            "wdref_check_dims": (C.c_int, [i32p]),
            "wdref_index_tables": (C.c_int, [i32p, P, P, P, P]),
            "wdref_gamma": (None, [C.c_int, P]),
            "wdref_hop": (None, [i32p, P, P, P, C.c_int]),
            "wdref_wilson": (None, [i32p, P, d, P, P, C.c_int]),
            "wdref_mdagm": (None, [i32p, P, d, P, P]),
            "wdref_hop_eo": (None, [i32p, P, P, P, C.c_int, C.c_int]),
            "wdref_mhat": (None, [i32p, P, d, P, P, C.c_int]),
            "wdref_mhatdag_mhat": (None, [i32p, P, d, P, P]),
            "wdref_cg": (C.c_int, [i32p, P, d, C.c_int, P, P, d, C.c_int,
                                   C.POINTER(C.c_int), C.POINTER(d), P]),
            "wdref_plaquette": (d, [i32p, P]),
            "wdref_gauge_action": (d, [i32p, P, d]),
            "wdref_gauge_force": (None, [i32p, P, d, P]),
            "wdref_fermion_force_xy": (None, [i32p, P, P, P, d, P]),
            "wdref_fermion_force": (C.c_int, [i32p, P, d, C.c_int, P, d, C.c_int, P,
                                              C.POINTER(C.c_int)]),
            "wdref_fermion_action": (d, [i32p, P, d, C.c_int, P, d, C.c_int,
                                         C.POINTER(C.c_int)]),
            "wdref_expi": (None, [P, d, P]),
            "wdref_philox4x32_10": (None, [P, P, P]),
            "wdref_normal_pair": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_uint32, P]),
            "wdref_uniform": (d, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                  C.c_uint32]),
            "wdref_draw_momenta": (None, [i32p, C.c_uint64, C.c_uint32, P]),
            "wdref_draw_chi": (None, [C.c_long, C.c_uint64, C.c_uint32, P]),
            "wdref_kinetic": (d, [i32p, P]),
            "wdref_md_force": (C.c_int, [i32p, P, d, d, C.c_int, P, d, C.c_int, P,
                                         C.POINTER(C.c_int)]),
            "wdref_leapfrog": (C.c_int, [i32p, P, P, d, d, C.c_int, P, d, C.c_int, d,
                                         C.c_int, C.POINTER(C.c_int)]),
            "wdref_hmc_trajectory": (C.c_int, [i32p, P, d, d, C.c_int, d, C.c_int,
                                               C.c_uint64, C.c_uint32, d, d, C.c_int, P]),
            "wdref_polyakov": (None, [i32p, P, P]),
            "wdref_point_propagator": (C.c_int, [i32p, P, d, i32p, d, C.c_int, P, C.POINTER(C.c_int)]),
            "wdref_pion_correlator": (None, [i32p, P, i32p, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _dims(dims):
    return (C.c_int32 * 4)(*[int(v) for v in dims])


def _p(a):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def volume(dims):
    return int(np.prod(dims))


def index_tables(dims):
    """nb [V][8] (x+mu, x-mu per mu), cb [V], par [V], eo_lex [2][Vh]."""
    V = volume(dims)
    nb = np.zeros((V, 8), np.int32)
    cb = np.zeros(V, np.int32)
    par = np.zeros(V, np.uint8)
    eo = np.zeros((2, V // 2), np.int32)
    rc = lib().wdref_index_tables(_dims(dims), _p(nb), _p(cb), _p(par), _p(eo))
    if rc:
        raise ValueError(f"bad lattice dims {dims}")
    return nb, cb, par, eo


def gamma(mu):
    """gamma_{mu+1} for mu = 0..3 (x,y,z,t); mu = 4 gives gamma_5."""
    g = np.zeros((4, 4), np.complex128)
    lib().wdref_gamma(mu, _p(g))
    return g


def hop(dims, U, psi, dagger=False):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().wdref_hop(_dims(dims), _p(U), _p(psi), _p(out), int(dagger))
    return out


def wilson(dims, U, kappa, psi, dagger=False):
    """M psi = psi - kappa H psi (or M^dag)."""
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().wdref_wilson(_dims(dims), _p(U), float(kappa), _p(psi), _p(out), int(dagger))
    return out


def mdagm(dims, U, kappa, psi):
    U, psi = _c128(U), _c128(psi)
    out = np.empty_like(psi)
    lib().wdref_mdagm(_dims(dims), _p(U), float(kappa), _p(psi), _p(out))
    return out


def hop_eo(dims, U, psi_par, out_parity, dagger=False):
    """Parity block of H (or H^dag): output on `out_parity`, input on the other."""
    U, psi_par = _c128(U), _c128(psi_par)
    out = np.empty_like(psi_par)
    lib().wdref_hop_eo(_dims(dims), _p(U), _p(psi_par), _p(out), int(out_parity), int(dagger))
    return out


def mhat(dims, U, kappa, psi_e, dagger=False):
    U, psi_e = _c128(U), _c128(psi_e)
    out = np.empty_like(psi_e)
    lib().wdref_mhat(_dims(dims), _p(U), float(kappa), _p(psi_e), _p(out), int(dagger))
    return out


def mhatdag_mhat(dims, U, kappa, psi_e):
    U, psi_e = _c128(U), _c128(psi_e)
    out = np.empty_like(psi_e)
    lib().wdref_mhatdag_mhat(_dims(dims), _p(U), float(kappa), _p(psi_e), _p(out))
    return out


def cg(dims, U, kappa, b, eo=False, tol=1e-10, maxiter=None, history=False):
    """CG on M^dag M (eo=False, full lattice) or Mhat^dag Mhat (eo=True, even
    sites).  Returns (x, iters, true_rel, converged[, hist])."""
    U, b = _c128(U), _c128(b)
    x = np.zeros_like(b)
    if maxiter is None:
        maxiter = 10 * b.size
    it = C.c_int(0)
    tr = C.c_double(0)
    hist = np.zeros(maxiter + 1) if history else None
    rc = lib().wdref_cg(_dims(dims), _p(U), float(kappa), int(eo), _p(b), _p(x), float(tol),
                        int(maxiter), C.byref(it), C.byref(tr),
                        _p(hist) if history else None)
    res = (x, it.value, tr.value, rc == 0)
    if history:
        return res + (hist[: it.value + 1],)
    return res


def plaquette(dims, U):
    return lib().wdref_plaquette(_dims(dims), _p(_c128(U)))


def gauge_action(dims, U, beta):
    return lib().wdref_gauge_action(_dims(dims), _p(_c128(U)), float(beta))


def gauge_force(dims, U, beta):
    U = _c128(U)
    F = np.empty_like(U)
    lib().wdref_gauge_force(_dims(dims), _p(U), float(beta), _p(F))
    return F


def fermion_force_xy(dims, U, X, Y, coef):
    U, X, Y = _c128(U), _c128(X), _c128(Y)
    F = np.empty_like(U)
    lib().wdref_fermion_force_xy(_dims(dims), _p(U), _p(X), _p(Y), float(coef), _p(F))
    return F


def fermion_force(dims, U, kappa, phi, eo=True, tol=1e-12, maxiter=100000):
    U, phi = _c128(U), _c128(phi)
    F = np.empty_like(U)
    it = C.c_int(0)
    lib().wdref_fermion_force(_dims(dims), _p(U), float(kappa), int(eo), _p(phi), float(tol),
                              int(maxiter), _p(F), C.byref(it))
    return F, it.value


def fermion_action(dims, U, kappa, phi, eo=True, tol=1e-12, maxiter=100000):
    it = C.c_int(0)
    s = lib().wdref_fermion_action(_dims(dims), _p(_c128(U)), float(kappa), int(eo),
                                   _p(_c128(phi)), float(tol), int(maxiter), C.byref(it))
    return s, it.value


def md_force(dims, U, beta, kappa, phi, eo=True, tol=1e-12, maxiter=100000):
    U, phi = _c128(U), _c128(phi)
    F = np.empty_like(U)
    it = C.c_int(0)
    lib().wdref_md_force(_dims(dims), _p(U), float(beta), float(kappa), int(eo), _p(phi),
                         float(tol), int(maxiter), _p(F), C.byref(it))
    return F, it.value


def expi(P, a):
    """exp(i a P) for a 3x3 complex matrix P (power series)."""
    P = _c128(P).reshape(3, 3)
    E = np.empty_like(P)
    lib().wdref_expi(_p(P), float(a), _p(E))
    return E


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().wdref_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normal_pair(seed, site, traj, tag, j):
    out = np.zeros(2)
    lib().wdref_normal_pair(seed, site, traj, tag, j, _p(out))
    return out


def uniform(seed, site, traj, tag, j):
    return lib().wdref_uniform(seed, site, traj, tag, j)


def draw_momenta(dims, seed, traj):
    P = np.zeros((volume(dims), 4, 3, 3), np.complex128)
    lib().wdref_draw_momenta(_dims(dims), int(seed), int(traj), _p(P))
    return P


def draw_chi(nsites, seed, traj):
    chi = np.zeros((nsites, 4, 3), np.complex128)
    lib().wdref_draw_chi(int(nsites), int(seed), int(traj), _p(chi))
    return chi


def kinetic(dims, P):
    return lib().wdref_kinetic(_dims(dims), _p(_c128(P)))


def leapfrog(dims, U, P, beta, kappa, phi, tau, nsteps, eo=True, tol=1e-12, maxiter=100000):
    """Integrates (U, P) in place copies; returns (U, P, cg_iters)."""
    U = _c128(U).copy()
    P = _c128(P).copy()
    it = C.c_int(0)
    lib().wdref_leapfrog(_dims(dims), _p(U), _p(P), float(beta), float(kappa), int(eo),
                         _p(_c128(phi)), float(tau), int(nsteps), float(tol), int(maxiter),
                         C.byref(it))
    return U, P, it.value


def hmc_trajectory(dims, U, beta, kappa, tau, nsteps, seed, traj, eo=True, tol_force=1e-10,
                   tol_h=1e-12, maxiter=100000):
    """Returns (U_after, dict of results); U is not modified."""
    U = _c128(U).copy()
    out = np.zeros(8)
    lib().wdref_hmc_trajectory(_dims(dims), _p(U), float(beta), float(kappa), int(eo),
                               float(tau), int(nsteps), int(seed), int(traj),
                               float(tol_force), float(tol_h), int(maxiter), _p(out))
    keys = ["dH", "accepted", "plaquette", "H_old", "H_new", "Sf_start", "cg_iters", "u"]
    r = dict(zip(keys, out.tolist()))
    r["accepted"] = bool(r["accepted"])
    r["cg_iters"] = int(r["cg_iters"])
    return U, r


def polyakov(dims, U):
    out = np.zeros(2)
    lib().wdref_polyakov(_dims(dims), _p(_c128(U)), _p(out))
    return complex(out[0], out[1])


def point_propagator(dims, U, kappa, src, tol=1e-12, maxiter=100000):
    """psi [12][V][4][3]: column 3*spin + colour solves M psi = point source
    at src (spin, colour); returns (psi, status, summed CG iterations)."""
    V = volume(dims)
    psi = np.zeros((12, V, 4, 3), np.complex128)
    it = C.c_int(0)
    st = lib().wdref_point_propagator(_dims(dims), _p(_c128(U)), float(kappa), _dims(src), float(tol),
                                      int(maxiter), _p(psi), C.byref(it))
    return psi, st, it.value


def pion_correlator(dims, psi, src):
    corr = np.zeros(dims[3])
    lib().wdref_pion_correlator(_dims(dims), _p(_c128(psi)), _dims(src), _p(corr))
    return corr
