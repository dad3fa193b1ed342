"""GPU parity of the index arithmetic and the hopping stencil (Sec. 3 kernel 1
and the neighbour routine) against the oracle: index tables bit-exact, FP64
stencil to 1e-12 relative, FP32 / FP16 to their rounding level."""
import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, empty_like_dev, host, maxabs_ratio, note, rel_err

pytestmark = pytest.mark.gpu

DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 4, 6), (4, 6, 2, 8), (8, 8, 8, 8)]


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


@pytest.mark.parametrize("dims", DIMS + [(12, 12, 12, 24), (16, 16, 16, 32)])
def test_device_tables_bit_exact(wd, oracle, dims):
    import torch
    note(f"device tables {dims}")
    V = li.volume(dims)
    lat = wd.Lattice(dims)
    nb = torch.zeros((V, 8), dtype=torch.int32, device="cuda")
    cb = torch.zeros(V, dtype=torch.int32, device="cuda")
    par = torch.zeros(V, dtype=torch.uint8, device="cuda")
    wd.wd_debug_device_tables(lat.ctx, nb, cb, par)
    onb, ocb, opar, _ = oracle.index_tables(dims)
    assert np.array_equal(host(nb), onb)
    assert np.array_equal(host(cb), ocb)
    assert np.array_equal(host(par), opar)
    lat.close()


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_fp64_parity_blocks(wd, oracle, dims, recon):
    note(f"dslash fp64 {dims} recon {recon}")
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=1001)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=recon)
    for out_par in (0, 1):
        psi = li.gaussian_spinor(V // 2, seed=7 + out_par)
        for dag in (0, 1):
            ref = oracle.hop_eo(dims, U, psi, out_par, dagger=bool(dag))
            out = empty_like_dev(psi)
            lat.dslash(out, dev(psi), wd.WD_EVEN if out_par == 0 else wd.WD_ODD, dag, wd.WD_F64)
            got = host(out)
            assert rel_err(got, ref) <= 1e-12, (out_par, dag, rel_err(got, ref))
            assert maxabs_ratio(got, ref) <= 1e-12
    lat.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_dslash_fp64_full_lattice(wd, oracle, dims):
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=3)
    psi = li.gaussian_spinor(V, seed=4)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U))
    for dag in (0, 1):
        out = empty_like_dev(psi)
        lat.dslash(out, dev(psi), wd.WD_FULL, dag, wd.WD_F64)
        assert rel_err(host(out), oracle.hop(dims, U, psi, dagger=bool(dag))) <= 1e-12
    lat.close()


# (relative 2-norm, max-abs ratio) bounds, about 2-2.5x the rounding each
# format shows on this lattice and field: relative 2-norm / largest component
# error over largest output component, measured on MI355X: F32 9.0e-8 /
# 1.25e-7, F16 2.5e-4 / 3.3e-4, F16L 4.0e-4 / 5.5e-4, F32L 2.0e-4 / 2.4e-4,
# F32R 8.7e-8 / 1.25e-7, F16R 2.5e-4 / 3.3e-4, I16 2.8e-5 / 2.7e-5, I16L
# 2.0e-4 / 2.4e-4.
SLOPPY_TOL = {"F32": (2e-7, 3e-7), "F16": (6e-4, 8e-4), "F16L": (9e-4, 1.4e-3), "F32L": (4.5e-4, 6e-4),
              "F32R": (2e-7, 3e-7), "F16R": (6e-4, 8e-4), "I16": (6e-5, 7e-5), "I16L": (4.5e-4, 6e-4),
              # 8-real FP32 links (measured: F32R8 2.7e-7 / 3.9e-7, F16R8 as F16)
              "F32R8": (6e-7, 9e-7), "F16R8": (6e-4, 8e-4)}


@pytest.mark.parametrize("prec", sorted(SLOPPY_TOL))
def test_dslash_sloppy_precisions(wd, oracle, prec):
    """I16 (int16 fixed point, per-site norm): quantisation step n/32767 per
    component, so about 1e-5 relative on Gaussian spinors -- well below
    FP16's 2^-11 relative rounding -- plus the FP32 link rounding."""
    tol, tol_max = SLOPPY_TOL[prec]
    dims = (6, 4, 4, 6)
    code = {"F32": wd.WD_F32, "F16": wd.WD_F16, "F16L": wd.WD_F16 | wd.WD_LINKS_F16,
            "F32L": wd.WD_F32 | wd.WD_LINKS_F16, "F32R": wd.WD_F32 | wd.WD_LINKS_R18,
            "F16R": wd.WD_F16 | wd.WD_LINKS_R18, "I16": wd.WD_I16,
            "I16L": wd.WD_I16 | wd.WD_LINKS_F16,
            "F32R8": wd.WD_F32 | wd.WD_LINKS_R8, "F16R8": wd.WD_F16 | wd.WD_LINKS_R8}[prec]
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=5)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U))
    psi = li.gaussian_spinor(V // 2, seed=6)
    for dag in (0, 1):
        ref = oracle.hop_eo(dims, U, psi, 0, dagger=bool(dag))
        out = empty_like_dev(psi)
        lat.dslash(out, dev(psi), wd.WD_EVEN, dag, code)
        got = host(out)
        e, m = rel_err(got, ref), maxabs_ratio(got, ref)
        note(f"dslash {prec} dag {dag}: rel err {e:.2e}, max-abs ratio {m:.2e}")
        assert e <= tol and m <= tol_max
    lat.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_mdagm_matches_oracle(wd, oracle, dims):
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=8)
    kappa = 0.155
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    pe = li.gaussian_spinor(V // 2, seed=9)
    out = empty_like_dev(pe)
    lat.mdagm(out, dev(pe), kappa, eo=1)
    assert rel_err(host(out), oracle.mhatdag_mhat(dims, U, kappa, pe)) <= 1e-12
    pf = li.gaussian_spinor(V, seed=10)
    out = empty_like_dev(pf)
    lat.mdagm(out, dev(pf), kappa, eo=0)
    assert rel_err(host(out), oracle.mdagm(dims, U, kappa, pf)) <= 1e-12
    lat.close()


def test_unit_gauge_free_field_plane_wave(wd):
    """U = 1: H e^{ipx} s = e^{ipx} sum_mu [2 cos p_mu - 2i g_mu sin p_mu] s
    (closed form, no oracle involved)."""
    from brute import GAMMA, sites
    dims = (4, 6, 4, 8)
    V = li.volume(dims)
    c = sites(dims)
    n = np.array([1, 2, 3, 5])
    p = 2 * np.pi * n / np.array(dims)
    rng = np.random.default_rng(0)
    s = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = np.exp(1j * (c @ p))[:, None, None] * s[None]
    K = sum(2 * np.cos(p[m]) * np.eye(4) - 2j * GAMMA[m] * np.sin(p[m]) for m in range(4))
    ref = np.exp(1j * (c @ p))[:, None, None] * (K @ s)[None]
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.unit_field(dims)))
    out = empty_like_dev(psi)
    lat.dslash(out, dev(psi), wd.WD_FULL, 0, wd.WD_F64)
    assert rel_err(host(out), ref) <= 1e-13
    lat.close()


def test_errors(wd):
    import torch
    with pytest.raises(wd.WDError) as e:
        wd.Lattice((4, 4, 5, 4))
    assert e.value.status == wd.WD_ERR_DIMS
    lat = wd.Lattice((4, 4, 4, 4))
    x = torch.zeros((128, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(wd.WDError) as e:
        lat.dslash(x, x.clone(), wd.WD_EVEN)
    assert e.value.status == wd.WD_ERR_STATE
    lat.gauge_load(dev(li.unit_field((4, 4, 4, 4))))
    # precision codes outside the formats: unknown base, int16 with 18-real links, two link flags
    for code in (4, wd.WD_I16 | wd.WD_LINKS_R18, wd.WD_F16 | wd.WD_LINKS_F16 | wd.WD_LINKS_R18):
        with pytest.raises(wd.WDError) as e:
            lat.dslash(x, x.clone(), wd.WD_EVEN, 0, code)
        assert e.value.status == wd.WD_ERR_ARG
    lat.close()


@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (8, 8, 8, 8)])
def test_pack_unpack_round_trip_bit_exact(wd, dims):
    """Canonical complex128 -> the internal FP64 structure-of-arrays layout ->
    canonical again gives the same bits, for parity fields (cb order) and full
    fields (lex order), several right-hand sides back to back: a solve that
    starts from x and stops before its first iteration returns x unchanged."""
    V = li.volume(dims)
    for eo, sites in ((1, V // 2), (0, V)):
        X0 = li.gaussian_spinor(sites, seed=31 + eo, nrhs=3)
        B = li.gaussian_spinor(sites, seed=41 + eo, nrhs=3)
        lat = wd.Lattice(dims)
        lat.gauge_load(dev(li.random_su3_field(dims, 0.5, seed=5)), recon=12)
        x = dev(X0)
        st, stats = lat.cg_solve(x, dev(B), 0.15, wd.solver_params(maxiter=0, eo=eo, initial_guess=1))
        assert st == wd.WD_ERR_NOCONV and all(s["iters"] == 0 for s in stats)
        got = host(x)
        assert np.array_equal(got.view(np.uint64), X0.view(np.uint64)), eo
        lat.close()


@pytest.mark.parametrize("eps", [0.5, 0.05, 0.0])
def test_eight_real_links(wd, oracle, eps):
    """8-real FP32 links against the oracle on a random field (eps 0.5), a
    field near the identity (eps 0.05: |a2|^2 + |a3|^2 ~ 1e-3 after the
    pivot, the division by it must not cost accuracy) and U = 1 (every link
    block-diagonal: reconstructed exactly, so the stencil equals the 12-real
    one value for value)."""
    dims = (8, 8, 8, 8)
    V = li.volume(dims)
    U = li.random_su3_field(dims, eps, seed=9) if eps > 0 else li.unit_field(dims)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    psi = li.gaussian_spinor(V // 2, seed=10)
    # (measured: FP32 spinors 2.9e-7 relative and 4.4e-7 max-abs at worst, FP16 as with 12-real links)
    for sp, tol in ((wd.WD_F32, 6e-7), (wd.WD_F16, 6e-4)):
        for dag in (0, 1):
            ref = oracle.hop_eo(dims, U, psi, 1, dagger=bool(dag))
            out8, out12 = empty_like_dev(psi), empty_like_dev(psi)
            lat.dslash(out8, dev(psi), wd.WD_ODD, dag, sp | wd.WD_LINKS_R8)
            lat.dslash(out12, dev(psi), wd.WD_ODD, dag, sp)
            g8, g12 = host(out8), host(out12)
            e8, e12, m8 = rel_err(g8, ref), rel_err(g12, ref), maxabs_ratio(g8, ref)
            note(f"8-real eps {eps} sp {sp} dag {dag}: rel {e8:.2e} (12-real {e12:.2e}), max-abs ratio {m8:.2e}")
            assert e8 <= tol and m8 <= 2 * tol
            if eps == 0.0:
                assert np.array_equal(g8, g12)
    lat.close()
