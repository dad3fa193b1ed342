"""Faces of a lattice cut along t (the paper's next step, running over
several GPUs, Sec. 4 end): the forward face (1 -+ g_t) psi of slice 0 and the
backward face U_t^dag (1 +- g_t) psi of slice Lt-1, applied to the output
sites of slices Lt-1 and 0, must give exactly the t-neighbour terms of the
hopping operator across the cut.  The oracle side isolates those terms: with
psi zero except on slice 0, the oracle's hopping block at the sites of slice
Lt-1 is the forward term across the cut alone (their other neighbours lie on
slices Lt-1 and Lt-2), and with psi zero except on slice Lt-1, at the sites
of slice 0 it is the backward term alone (Lt >= 4)."""
import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, empty_like_dev, host, note, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


def slice_of(dims):
    """t coordinate of each checkerboard index of a parity field."""
    Vh = li.volume(dims) // 2
    return np.arange(Vh) // (dims[0] * dims[1] * dims[2] // 2)


def expected(oracle, dims, U, psi, out_par, dag):
    Lt = dims[3]
    t = slice_of(dims)
    pf = np.where((t == 0)[:, None, None], psi, 0)
    pb = np.where((t == Lt - 1)[:, None, None], psi, 0)
    hf = oracle.hop_eo(dims, U, pf, out_par, dagger=bool(dag))
    hb = oracle.hop_eo(dims, U, pb, out_par, dagger=bool(dag))
    ref = np.zeros_like(psi)
    ref[t == Lt - 1] = hf[t == Lt - 1]
    ref[t == 0] = hb[t == 0]
    return ref


@pytest.mark.parametrize("prec,tol", [("F64", 1e-13), ("F32", 2e-6), ("F16", 4e-3), ("F16L", 5e-3),
                                      ("F32R", 2e-6)])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 6), (4, 6, 4, 8)])
def test_face_terms_equal_cut_terms_of_the_operator(wd, oracle, prec, tol, dims):
    code = {"F64": wd.WD_F64, "F32": wd.WD_F32, "F16": wd.WD_F16,
            "F16L": wd.WD_F16 | wd.WD_LINKS_F16, "F32R": wd.WD_F32 | wd.WD_LINKS_R18}[prec]
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=61)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    t = slice_of(dims)
    off = (t != 0) & (t != dims[3] - 1)
    for out_par in (0, 1):
        psi = li.gaussian_spinor(V // 2, seed=62 + out_par)
        for dag in (0, 1):
            note(f"faces {prec} {dims} parity {out_par} dagger {dag}")
            ref = expected(oracle, dims, U, psi, out_par, dag)
            out = empty_like_dev(psi)
            lat.faces_apply(out, dev(psi), wd.WD_EVEN if out_par == 0 else wd.WD_ODD, dag, code)
            got = host(out)
            assert np.all(got[off] == 0)
            err = rel_err(got, ref)
            assert err <= tol, (out_par, dag, err)
    lat.close()


def test_faces_plus_interior_is_the_stencil(wd, oracle):
    """The face terms and the oracle's stencil on psi with the slices that
    feed them zeroed add up, on the boundary slices, to the full stencil (an
    FP64 check that no term across the cut is missed or doubled)."""
    dims = (4, 4, 4, 6)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=63)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=18)
    psi = li.gaussian_spinor(V // 2, seed=64)
    out = empty_like_dev(psi)
    lat.faces_apply(out, dev(psi), wd.WD_ODD, 0, wd.WD_F64)
    full = oracle.hop_eo(dims, U, psi, 1)
    t = slice_of(dims)
    Lt = dims[3]
    # interior part on slice Lt-1: everything but its neighbours on slice 0
    inner_top = oracle.hop_eo(dims, U, np.where((t == 0)[:, None, None], 0, psi), 1)
    inner_bot = oracle.hop_eo(dims, U, np.where((t == Lt - 1)[:, None, None], 0, psi), 1)
    got = host(out)
    assert rel_err(got[t == Lt - 1] + inner_top[t == Lt - 1], full[t == Lt - 1]) <= 1e-13
    assert rel_err(got[t == 0] + inner_bot[t == 0], full[t == 0]) <= 1e-13
    lat.close()


def test_face_errors(wd):
    import torch
    dims = (4, 4, 4, 4)
    lat = wd.Lattice(dims)
    x = torch.zeros((128, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(wd.WDError) as e:
        lat.faces_apply(x, x.clone(), wd.WD_EVEN)
    assert e.value.status == wd.WD_ERR_STATE
    lat.gauge_load(dev(li.unit_field(dims)))
    for par, code in ((wd.WD_FULL, wd.WD_F64), (wd.WD_EVEN, wd.WD_I16), (wd.WD_EVEN, 4)):
        with pytest.raises(wd.WDError) as e:
            wd.wd_faces_apply(lat.ctx, x, x.clone(), par, 0, code)
        assert e.value.status == wd.WD_ERR_ARG
    with pytest.raises(ValueError):
        lat.faces_apply(x[:64], x.clone(), wd.WD_EVEN)
    lat.close()


def test_bench_faces_runs(wd):
    dims = (8, 8, 8, 8)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.unit_field(dims)))
    for code in (wd.WD_F64, wd.WD_F32, wd.WD_F16):
        pm, am, pb, ab = wd.wd_bench_faces(lat.ctx, code, iters=3)
        assert pm > 0 and am > 0 and pb > 0 and ab > 0
    lat.close()
