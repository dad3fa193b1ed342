"""Parity at the sizes the benchmark runs (Sec. 3 kernel 1 inside the CG of
eq. 3): lattices with several z- and t-planes per XCD, so that every tile
order's plane-within-slab terms are non-zero, and twelve right-hand sides, so
that the RHS-group index of every launch shape is exercised.

* every launch shape of the parity stencil gives the default shape's bits
  (compared on the device), and one shape per tile order is compared with the
  oracle element by element;
* the autotuner rejects no candidate at 16^3 x 32 with 12 RHS (FP16 and FP64);
* the tuned 12-RHS FP16 solve at 16^3 x 32 meets 1e-10 by the oracle's
  operator for every RHS and equals the default-shape solve bit for bit;
* at 32^3 x 64, the launch shapes of the committed MI355X shape table are
  re-verified by the tuner against the reference shape bit for bit, and each
  of their plain sweeps is compared with the oracle (FP64 element by element,
  FP16 at its rounding level).
"""
import os
import shutil

import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, empty_like_dev, host, maxabs_ratio, note, rel_err

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_1207_2223_amd", "tune_mi355x.txt")
NRHS = 12
F64_SHAPES = [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4), (2, 4)]
SLOPPY_SHAPES = [(nr, rl) for rl in (1, 2, 4) for nr in (1, 2, 3, 4)]
STRIPES = {0: 0, 1: 0, 2: 1, 3: 2, 4: 4, 5: 1, 6: 1, 7: 1}


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


def order_ok(dims, spb, remap):
    """Whether tile order `remap` applies to tiles of spb sites (the slab
    orders need the slab extent divisible by 8 and whole tiles per plane and
    stripe)."""
    if remap < 2:
        return True
    plane = dims[0] // 2 * dims[1]
    slab = dims[3] if remap in (5, 6) else dims[2]
    return slab % 8 == 0 and plane % spb == 0 and (plane // spb) % STRIPES[remap] == 0


def all_shapes(dims, f64):
    """Every launch shape of the FP64 or the FP16 (FP32 12-real links)
    stencil on this lattice, the LDS-staged and t-walking ones (every block
    size that tiles a plane) included."""
    from test_gpu_tune import lds_candidates, tw_candidates
    out = []
    for nr, rl in (F64_SHAPES if f64 else SLOPPY_SHAPES):
        for block in (64, 128, 256):
            for remap in range(8):
                if order_ok(dims, block // rl, remap):
                    out.append((block, nr, rl, remap, 0))
    code = 0 if f64 else 2
    return out + lds_candidates(dims, code, NRHS) + tw_candidates(dims, code, NRHS, blocks=(64, 128, 256))


def bits(t):
    import torch
    return torch.view_as_real(t).view(torch.int64)


def same_bits(a, b):
    import torch
    return torch.equal(bits(a), bits(b))


def tiled_field(dims, eps, seed, tile=8):
    """A periodic gauge field made of copies of a random 8^4 field: cheap to
    draw at 32^3 x 64, and any field is as good as another for parity."""
    small = li.random_su3_field((tile,) * 4, eps, seed=seed).reshape(tile, tile, tile, tile, 4, 3, 3)
    reps = (dims[3] // tile, dims[2] // tile, dims[1] // tile, dims[0] // tile, 1, 1, 1)
    return np.ascontiguousarray(np.tile(small, reps).reshape(li.volume(dims), 4, 3, 3))


@pytest.mark.parametrize("dims", [(16, 16, 16, 32), (32, 32, 16, 16)])
def test_every_launch_shape_and_tile_order(wd, oracle, dims):
    """(16,16,16,32): 2 z-planes and 4 t-planes per XCD; (32,32,16,16): 512
    sites per plane (the 32^3 x 64 plane, so 4 y-stripes apply) with 2 z- and
    2 t-planes per XCD.  The FP16 shapes include the LDS-staged kernel (4, 8,
    16 t-planes per work-group, 1 and 2 RHS per lane) and the t-walking kernel
    with the t neighbours in registers (4, 8, 16 t-planes, 1 to 3 RHS per
    lane, tiles of 64, 128 and 256 sites)."""
    import torch
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=1201)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    psi = li.gaussian_spinor(V // 2, seed=1202, nrhs=NRHS)
    d_in = dev(psi)
    for dag in (0, 1):
        ref = np.stack([oracle.hop_eo(dims, U, psi[j], 1, dagger=bool(dag)) for j in range(NRHS)])
        for f64 in (True, False):
            code = wd.WD_F64 if f64 else wd.WD_F16
            base = torch.empty_like(d_in)
            wd.wd_dslash_shaped(lat.ctx, base, d_in, wd.WD_ODD, dag, code, None)
            got = host(base)
            e, m = rel_err(got, ref), maxabs_ratio(got, ref)
            note(f"{dims} dag {dag} {'F64' if f64 else 'F16'} default shape vs oracle: rel {e:.2e} maxabs {m:.2e}")
            if f64:
                assert e <= 1e-12 and m <= 1e-12
            else:
                assert e <= 6e-4 and m <= 3e-3
            shapes = all_shapes(dims, f64)
            orders = sorted({s[3] for s in shapes})
            assert orders == list(range(8 if f64 else 14))
            checked = set()
            out = torch.empty_like(d_in)
            for shape in shapes:
                # (the library poisons its internal output before each sweep,
                # so a shape that skipped sites would leave NaNs here)
                wd.wd_dslash_shaped(lat.ctx, out, d_in, wd.WD_ODD, dag, code, shape)
                assert same_bits(out, base), (dims, dag, code, shape)
                # one shape per tile order with several RHS per group, element by element
                if f64 and shape[3] not in checked and shape[1] * shape[2] > 1:
                    checked.add(shape[3])
                    g = host(out)
                    assert rel_err(g, ref) <= 1e-12 and maxabs_ratio(g, ref) <= 1e-12, shape
            if f64:
                assert checked == set(orders)
            note(f"{dims} dag {dag} {'F64' if f64 else 'F16'}: {len(shapes)} shapes, tile orders {orders}")
    lat.close()


@pytest.mark.parametrize("prec", ["F16", "F64"])
def test_tuner_rejects_nothing_at_16c32_12rhs(wd, prec):
    from test_gpu_tune import _expected_candidates, nt_extra
    dims = (16, 16, 16, 32)
    code = wd.WD_F16 if prec == "F16" else wd.WD_F64
    U = li.random_su3_field(dims, 0.5, seed=1203)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    rows = wd.wd_tune(lat.ctx, NRHS, code)
    for r in rows:
        # (the best shape is retried with 7 work-group caps unless it is LDS-staged)
        want = _expected_candidates(dims, code, NRHS) - (7 if 8 <= r["remap"] <= 10 else 0) + nt_extra(code, r)
        note(f"{prec} {r['sweep']}: block {r['block']} nr {r['nr']} rl {r['rl']} remap {r['remap']} "
             f"occ {r['occ']}; {r['candidates']} candidates, {r['rejected']} rejected")
        assert r["source"] == "timed" and r["candidates"] == want and r["rejected"] == 0
    lat.close()


def test_tuned_12rhs_f16_solve_at_16c32(wd, oracle):
    dims = (16, 16, 16, 32)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=li.config_seed(2))
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    wd.wd_tune(lat.ctx, NRHS, wd.WD_F16)
    wd.wd_tune(lat.ctx, NRHS, wd.WD_F64)
    B = li.gaussian_spinor(V // 2, seed=2002, nrhs=NRHS)
    kap = [0.155] * NRHS
    X0, X1 = empty_like_dev(B), empty_like_dev(B)
    s1, st1 = lat.cg_solve(X1, dev(B), kap, wd.solver_params(prec=wd.WD_F16, delta=0.01, tuned=1))
    s0, st0 = lat.cg_solve(X0, dev(B), kap, wd.solver_params(prec=wd.WD_F16, delta=0.01, tuned=0))
    assert s0 == wd.WD_OK and s1 == wd.WD_OK
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    assert np.array_equal(host(X0), host(X1))
    Xh = host(X1)
    for j in range(NRHS):
        r = np.linalg.norm(B[j] - oracle.mhatdag_mhat(dims, U, kap[j], Xh[j])) / np.linalg.norm(B[j])
        note(f"rhs {j}: {st1[j]['iters']} iterations, oracle true residual {r:.3e}")
        assert r <= 1.01e-10
    lat.close()


def _table_rows(dims, nrhs):
    rows = []
    for line in open(TABLE):
        f = line.split()
        if len(f) < 15 or tuple(int(v) for v in f[:4]) != tuple(dims) or int(f[4]) != nrhs:
            continue
        sp, lk, dag, epi = (int(v) for v in f[5:9])
        rows.append(dict(sp=sp, lk=lk, dag=dag, epi=epi, shape=tuple(int(v) for v in f[9:14])))
    return rows


def test_shape_table_at_32c64(wd, oracle, tmp_path, monkeypatch):
    import torch
    dims = (32, 32, 32, 64)
    rows = _table_rows(dims, NRHS)
    assert rows, "no 12-RHS rows for 32^3 x 64 in the shape table"
    V = li.volume(dims)
    note("32^3 x 64: drawing the tiled gauge field")
    U = tiled_field(dims, 0.5, seed=1204)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    # 1) the tuner re-verifies every cached shape bit for bit (all four sweeps)
    cache = tmp_path / "table.txt"
    shutil.copy(TABLE, cache)
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    for code in (wd.WD_F16, wd.WD_F64):
        for r in wd.wd_tune(lat.ctx, NRHS, code):
            note(f"table {r['sweep']} sp {r['sp']}: remap {r['remap']} occ {r['occ']} -> {r['source']}")
            assert r["source"] == "cache-verified" and r["rejected"] == 0
    # 2) the plain sweeps of the table's shapes against the oracle
    psi = li.gaussian_spinor(V // 2, seed=1205, nrhs=NRHS)
    d_in = dev(psi)
    out = torch.empty_like(d_in)
    for dag in (0, 1):
        note(f"32^3 x 64: oracle D_oe (dagger {dag}) on {NRHS} RHS")
        ref = np.stack([oracle.hop_eo(dims, U, psi[j], 1, dagger=bool(dag)) for j in range(NRHS)])
        for row in rows:
            if row["epi"] != 0 or row["dag"] != dag:
                continue
            code = wd.WD_F64 if row["sp"] == 0 else wd.WD_F16
            wd.wd_dslash_shaped(lat.ctx, out, d_in, wd.WD_ODD, dag, code, row["shape"])
            g = host(out)
            e, m = rel_err(g, ref), maxabs_ratio(g, ref)
            note(f"table shape {row['shape']} sp {row['sp']} dag {dag}: rel {e:.2e} maxabs {m:.2e}")
            if row["sp"] == 0:
                assert e <= 1e-12 and m <= 1e-12
            else:
                assert e <= 6e-4 and m <= 3e-3
    lat.close()
