"""The binding refuses a tensor whose size does not match the lattice (eo or
full, parity), a solution buffer of another shape than its source, and a
tensor on the CPU or on another device, before any device pointer reaches the
library.  Runs without a GPU: a context is registered by hand, as wd_create
would record it, and no library call is made."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1207_2223_amd import wd

DIMS = (4, 4, 4, 8)
V = int(np.prod(DIMS))
Vh = V // 2
FAKE = 0x5EED0


@pytest.fixture()
def ctx():
    h = C.c_void_p(FAKE)
    wd._CTX[FAKE] = wd._CtxInfo(DIMS, device=0)
    yield h
    wd._CTX.pop(FAKE, None)


def c128(*shape):
    return torch.zeros(shape, dtype=torch.complex128)


def params(eo):
    p = wd.wd_solver_params()
    p.tol, p.maxiter, p.prec_sloppy, p.eo, p.delta, p.poll = 1e-10, 100, wd.WD_F64, eo, 0.1, 8
    return p


def refused(fn, *args, match):
    with pytest.raises(ValueError, match=match):
        fn(*args)


def test_unknown_context_is_refused():
    refused(wd.wd_dslash, C.c_void_p(12345), c128(Vh, 4, 3), c128(Vh, 4, 3), wd.WD_EVEN,
            match="unknown context")


def test_stencil_sizes_follow_the_parity(ctx):
    # a parity sweep takes Vh sites, a full one V sites
    refused(wd.wd_dslash, ctx, c128(Vh - 1, 4, 3), c128(Vh, 4, 3), wd.WD_EVEN, match="out has shape")
    refused(wd.wd_dslash, ctx, c128(Vh, 4, 3), c128(Vh, 4, 3), wd.WD_FULL, match="out has shape")
    refused(wd.wd_dslash, ctx, c128(V, 4, 3), c128(Vh, 4, 3), wd.WD_FULL, match="in has shape")
    # right sizes, but host memory
    refused(wd.wd_dslash, ctx, c128(Vh, 4, 3), c128(Vh, 4, 3), wd.WD_ODD, match="CUDA")
    refused(wd.wd_mdagm, ctx, c128(V, 4, 3), c128(V, 4, 3), 0.15, 1, match="out has shape")
    refused(wd.wd_mdagm, ctx, c128(V, 4, 3), c128(V, 4, 3), 0.15, 0, match="CUDA")


def test_solver_buffers_match_the_source_and_the_lattice(ctx):
    refused(wd.wd_cg_solve, ctx, c128(2, Vh, 4, 3), c128(3, Vh, 4, 3), 0.15, params(1),
            match="must match")
    refused(wd.wd_cg_solve, ctx, c128(2, V, 4, 3), c128(2, V, 4, 3), 0.15, params(1),
            match="phi has shape")
    refused(wd.wd_cg_solve, ctx, c128(2, Vh, 4, 3), c128(2, Vh, 4, 3), 0.15, params(0),
            match="phi has shape")
    refused(wd.wd_cg_solve, ctx, c128(2, Vh, 4, 3), c128(2, Vh, 4, 3), 0.15, params(1), match="CUDA")


def test_session_buffers_follow_the_session(ctx):
    sess = C.c_void_p(FAKE + 1)
    wd._SESS[FAKE + 1] = (wd._CTX[FAKE], 1)
    try:
        refused(wd.wd_session_add, sess, c128(3, V, 4, 3), [0.15] * 3, match="phi has shape")
        refused(wd.wd_session_take, sess, 0, c128(2, Vh, 4, 3), match="x has shape")
        refused(wd.wd_session_take, sess, 0, c128(Vh, 4, 3), match="CUDA")
    finally:
        wd._SESS.pop(FAKE + 1, None)
    refused(wd.wd_session_take, sess, 0, c128(Vh, 4, 3), match="unknown session")


def test_gauge_and_hmc_fields(ctx):
    refused(wd.wd_gauge_load, ctx, c128(Vh, 4, 3, 3), match="U has shape")
    refused(wd.wd_hmc_draw, ctx, c128(V, 4, 3, 3), c128(V, 4, 3), 1, 0, match="chi has shape")
    refused(wd.wd_md_force, ctx, c128(V, 4, 3, 3), c128(V, 4, 3, 3), c128(V, 4, 3), 0.15, 5.6,
            match="phi has shape")
    refused(wd.hmc_trajectory, ctx, c128(V - 2, 4, 3, 3), None, match="U has shape")
    refused(wd.wd_plaquette, ctx, c128(V, 4, 3, 3), match="CUDA")
    refused(wd.wd_point_propagator, ctx, c128(12, Vh, 4, 3), (0, 0, 0, 0), 0.15, match="psi has shape")
    refused(wd.wd_faces_apply, ctx, c128(V, 4, 3), c128(Vh, 4, 3), wd.WD_EVEN, match="out has shape")


def test_debug_tables_sizes_and_types(ctx):
    refused(wd.wd_debug_device_tables, ctx, torch.zeros(8 * V, dtype=torch.int64),
            torch.zeros(V, dtype=torch.int32), torch.zeros(V, dtype=torch.uint8), match="nb must be")
    refused(wd.wd_debug_device_tables, ctx, torch.zeros(8 * V, dtype=torch.int32),
            torch.zeros(V - 1, dtype=torch.int32), torch.zeros(V, dtype=torch.uint8), match="cb must be")


def test_device_index_must_match():
    info = wd._CtxInfo(DIMS, device=1)

    class OnDev0:  # stands for a CUDA tensor on device 0
        is_cuda = True
        device = torch.device("cuda", 0)

    with pytest.raises(ValueError, match="on device 0, the context on device 1"):
        wd._on_device(OnDev0(), info, "x")
