"""Autotuner: every launch shape of every sweep produces bitwise-identical
vectors and norm partials (the tuner rejects any that does not; none may be
rejected), and a solve with tuned shapes equals the default-shape solve bit
for bit."""
import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, empty_like_dev, host, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


def lds_limit():
    """LDS bytes a work-group may use on this device (the library asks the
    runtime the same)."""
    import torch
    return int(torch.cuda.get_device_properties(0).shared_memory_per_block)


def lds_candidates(dims, code, nrhs):
    """The LDS-staged shapes (tile orders 8, 9, 10: 4, 8, 16 t-planes per
    work-group; 256 threads, 1 lane per site, 1 or 2 RHS per lane): FP16
    spinors with FP32 or FP16 12-real links, FP32 spinors with FP32 12-real
    links (1 RHS per lane), where a plane of one parity has a multiple of 64
    sites up to 512, Lz % 8 == 0, Lt divisible by the chunk and three input
    planes of the lane's RHS fit in LDS."""
    base, links = code & 0xF, code & 0x70
    if base == 2 and links in (0, 0x10):
        nrs, sb = (1, 2), 52
    elif base == 1 and links == 0:
        nrs, sb = (1,), 96
    else:
        return []
    S = dims[0] // 2 * dims[1]
    out = []
    for nr in nrs:
        if nr > 2 * nrhs and nr != 1:
            continue
        for rm, tc in ((8, 4), (9, 8), (10, 16)):
            if S % 64 == 0 and S <= 512 and dims[2] % 8 == 0 and dims[3] % tc == 0 and \
                    3 * nr * S * sb <= lds_limit():
                out.append((256, nr, 1, rm, 0))
    return out


def tw_candidates(dims, code, nrhs, blocks=None):
    """The t-walking shapes (tile orders 11, 12, 13: 4, 8, 16 t-planes per
    work-group, the t neighbours held in registers; one lane per site, 1 to 3
    RHS per lane): FP16 spinors with FP32 or FP16 12-real links, where a plane
    of one parity holds whole tiles of the block's sites, Lz % 8 == 0 and Lt
    is divisible by the chunk.  The tuner tries the largest block of 256,
    128, 64 that divides a plane; `blocks` lists others to include."""
    base, links = code & 0xF, code & 0x70
    if base != 2 or links not in (0, 0x10):
        return []
    S = dims[0] // 2 * dims[1]
    tb = 256 if S % 256 == 0 else (128 if S % 128 == 0 else 64)
    out = []
    for b in (blocks or (tb,)):
        if S % b != 0 or dims[2] % 8 != 0:
            continue
        for nr in (1, 2, 3):
            if nr > 2 * nrhs and nr != 1:
                continue
            for rm, tc in ((11, 4), (12, 8), (13, 16)):
                if dims[3] % tc == 0:
                    out.append((b, nr, 1, rm, 0))
    return out


def nt_extra(code, row):
    """1 if the tuner retried the sweep's best shape with its links loaded
    non-temporally: FP16 or FP32 spinors with FP32 12- or 8-real links, or
    FP64 spinors with FP64 12-real links; the register-tiled kernel (orders
    0-7), one lane per site, 1 or 2 RHS per lane."""
    fmt = (row["lk"] in (2, 5) and row["sp"] in (1, 2)) or (row["lk"] == 1 and row["sp"] == 0)
    return int(fmt and row["rl"] == 1 and row["nr"] in (1, 2) and row["remap"] < 8)


def _expected_candidates(dims, code, nrhs):
    """The tuner's candidate count: block {64,128,256} x RHS per lane x lanes
    per site x tile order {plain, XCD round-robin, z-slab with 1, 2, 4
    y-stripes, t-slab walked t-fastest in two orders, z-slab with the RHS
    groups outermost}, where the z-slab orders need Lz % 8 == 0, the t-slab
    orders Lt % 8 == 0, and all a whole number of tiles per plane and per
    stripe; the LDS-staged and t-walking shapes where they apply; then the
    best of these with a cap of 2..8 work-groups per CU (7 more, unless the
    best is an LDS-staged shape, which takes no cap: then the count is 7
    less)."""
    few = (code & 0xF) == 0 or (code & 0x40)  # FP64, or 8-real links: 1 or 2 RHS per lane
    shapes = [(1, 1), (2, 1), (1, 2), (2, 2), (1, 4), (2, 4)] if few else \
        [(nr, rl) for rl in (1, 2, 4) for nr in (1, 2, 3, 4)]
    plane = dims[0] // 2 * dims[1]
    n = 0
    for nr, rl in shapes:
        if nr * rl > 2 * nrhs and not (nr == 1 and rl == 1):
            continue
        for b in (64, 128, 256):
            spb = b // rl
            for rm, ns in ((0, 0), (1, 0), (2, 1), (3, 2), (4, 4), (5, 1), (6, 1), (7, 1)):
                slab = dims[3] if rm in (5, 6) else dims[2]
                if rm >= 2 and not (slab % 8 == 0 and plane % spb == 0 and (plane // spb) % ns == 0):
                    continue
                n += 1
    return n + len(lds_candidates(dims, code, nrhs)) + len(tw_candidates(dims, code, nrhs)) + 7


@pytest.mark.parametrize("prec", ["F64", "F32", "F16", "F16L", "F16R", "F16R8", "I16"])
@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (16, 8, 8, 4), (16, 16, 8, 4), (8, 8, 4, 8)])
def test_tuner_all_shapes_bitwise_and_tuned_solve_identical(wd, oracle, prec, dims):
    """(6,4,4,6): Vh = 288, a ragged last tile for every block size;
    (16,8,8,4): Lz divisible by 8, so the z-slab tile order is a candidate;
    (16,16,8,4): 128 cb sites per plane, so the z-slab order in 2 and 4
    y-stripes is a candidate too; (8,8,4,8): Lt divisible by 8, so the
    t-slab orders are candidates."""
    code = {"F64": wd.WD_F64, "F32": wd.WD_F32, "F16": wd.WD_F16,
            "F16L": wd.WD_F16 | wd.WD_LINKS_F16, "F16R": wd.WD_F16 | wd.WD_LINKS_R18,
            "F16R8": wd.WD_F16 | wd.WD_LINKS_R8,
            "I16": wd.WD_I16}[prec]
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=41)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    nrhs = 5
    rows = wd.wd_tune(lat.ctx, nrhs, code)
    for r in rows:
        want = _expected_candidates(dims, code, nrhs) - (7 if 8 <= r["remap"] <= 10 else 0) + nt_extra(code, r)
        assert r["candidates"] == want, (r, want)
    for r in rows:
        note(f"{prec} {r['sweep']}: block {r['block']} nr {r['nr']} rl {r['rl']} remap {r['remap']} "
             f"occ {r['occ']} {r['candidates']} candidates, {r['rejected']} rejected")
        assert r["rejected"] == 0 and r["candidates"] > 1
        assert r["occ"] == 0 or 2 <= r["occ"] <= 8
        assert r["lnt"] in (0, 1) and (r["lnt"] == 0 or nt_extra(code, r))
    if code != wd.WD_F64:
        wd.wd_tune(lat.ctx, nrhs, wd.WD_F64)
    B = li.gaussian_spinor(V // 2, seed=42, nrhs=nrhs)
    kap = [0.15, 0.152, 0.154, 0.156, 0.157]
    X0 = empty_like_dev(B)
    X1 = empty_like_dev(B)
    s0, st0 = lat.cg_solve(X0, dev(B), kap, wd.solver_params(prec=code, tuned=0))
    s1, st1 = lat.cg_solve(X1, dev(B), kap, wd.solver_params(prec=code, tuned=1))
    assert s0 == wd.WD_OK and s1 == wd.WD_OK
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    assert np.array_equal(host(X0), host(X1))
    # and the result is a solution by the oracle's operator
    Xh = host(X1)
    for j in range(nrhs):
        r = B[j] - oracle.mhatdag_mhat(dims, U, kap[j], Xh[j])
        assert np.linalg.norm(r) / np.linalg.norm(B[j]) <= 1.01e-10
    lat.close()


def test_bench_dslash_runs(wd):
    dims = (8, 8, 8, 8)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.unit_field(dims)))
    for epi in (0, 1, 2):
        ms, by = wd.wd_bench_dslash(lat.ctx, 3, wd.WD_F16, epi=epi, iters=3, tuned=0)
        assert ms > 0 and by > 0
    lat.close()


def test_cached_shapes_with_work_group_cap(wd, tmp_path, monkeypatch):
    """Shapes read from the tuning cache file, here with a cap of 3 and 5
    work-groups per CU (and one line in the older format without the cap
    field), drive a tuned solve that equals the default-shape solve bit for
    bit."""
    dims = (8, 8, 8, 8)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=51)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    key = "8 8 8 8 3 2 2"  # dims, nrhs 3, FP16 spinors, FP32 12-real links
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key} 0 0 128 2 1 1 3 1.0\n"     # D_oe: block 128, nr 2, rl 1, cap 3
                     f"{key} 0 1 256 1 2 1 5 1.0\n"     # xpay: block 256, nr 1, rl 2, cap 5
                     f"{key} 1 0 64 3 1 0 1.0\n"        # D_oe^dag: older line, no cap
                     f"{key} 1 2 128 1 1 1 4 1.0\n")    # CG update: cap 4
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    rows = wd.wd_tune(lat.ctx, 3, wd.WD_F16)
    assert [r["occ"] for r in rows] == [3, 5, 0, 4]
    assert [r["candidates"] for r in rows] == [1, 1, 1, 1]
    assert [r["source"] for r in rows] == ["cache-verified"] * 4 and all(r["rejected"] == 0 for r in rows)
    B = li.gaussian_spinor(V // 2, seed=52, nrhs=3)
    kap = [0.15, 0.153, 0.156]
    X0 = empty_like_dev(B)
    X1 = empty_like_dev(B)
    s0, st0 = lat.cg_solve(X0, dev(B), kap, wd.solver_params(prec=wd.WD_F16, tuned=0))
    s1, st1 = lat.cg_solve(X1, dev(B), kap, wd.solver_params(prec=wd.WD_F16, tuned=1))
    assert s0 == wd.WD_OK and s1 == wd.WD_OK
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    assert np.array_equal(host(X0), host(X1))
    lat.close()


@pytest.mark.parametrize("prec", ["F16", "F64", "F32R8", "F16R8"])
def test_cached_shapes_with_nontemporal_links(wd, tmp_path, monkeypatch, prec):
    """Cache lines with the trailing non-temporal-links field, for every link
    format that has a non-temporal variant (FP32 12-real with FP16 spinors,
    FP64 12-real with FP64 spinors, FP32 8-real with FP32 and FP16 spinors):
    the solve with those shapes runs the non-temporal instances (their link
    format codes 6, 7, 8 in the timing report's kernel names) and equals the
    default-shape solve bit for bit."""
    code, sp, lk, lkn = {"F16": (wd.WD_F16, 2, 2, 6), "F64": (wd.WD_F64, 0, 1, 7),
                         "F32R8": (wd.WD_F32 | wd.WD_LINKS_R8, 1, 5, 8),
                         "F16R8": (wd.WD_F16 | wd.WD_LINKS_R8, 2, 5, 8)}[prec]
    dims = (8, 8, 8, 8)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=53)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(U), recon=12)
    key = f"8 8 8 8 2 {sp} {lk}"  # dims, nrhs 2, spinor and link format
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key} 0 0 128 2 1 1 3 1.0 1\n"   # D_oe: nr 2, cap 3, non-temporal links
                     f"{key} 0 1 256 1 2 1 0 1.0\n"     # xpay: rl 2 (no lnt field)
                     f"{key} 1 0 64 1 1 1 0 1.0 1\n"    # D_oe^dag: nr 1, block 64, non-temporal links
                     f"{key} 1 2 128 1 1 1 4 1.0 1\n")  # CG update: cap 4, non-temporal links
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    rows = wd.wd_tune(lat.ctx, 2, code)
    assert [r["lnt"] for r in rows] == [1, 0, 1, 1]
    assert [r["source"] for r in rows] == ["cache-verified"] * 4 and all(r["rejected"] == 0 for r in rows)
    B = li.gaussian_spinor(V // 2, seed=54, nrhs=2)
    kap = [0.15, 0.156]
    X0 = empty_like_dev(B)
    X1 = empty_like_dev(B)
    s0, st0 = lat.cg_solve(X0, dev(B), kap, wd.solver_params(prec=code, tuned=0))
    wd.wd_timing_enable(lat.ctx, True)
    s1, st1 = lat.cg_solve(X1, dev(B), kap, wd.solver_params(prec=code, tuned=1))
    names = set(wd.wd_timing_report(lat.ctx))
    wd.wd_timing_read(lat.ctx)
    wd.wd_timing_enable(lat.ctx, False)
    assert f"dslash_kernel<{sp}, {lkn}, 2, 1, false, 0>" in names, names
    assert f"dslash_kernel<{sp}, {lkn}, 1, 1, true, 2>" in names, names
    assert s0 == wd.WD_OK and s1 == wd.WD_OK
    assert [s["iters"] for s in st0] == [s["iters"] for s in st1]
    assert np.array_equal(host(X0), host(X1))
    lat.close()


def test_invalid_launch_shapes_are_refused_before_any_launch(wd):
    """wd_dslash_shaped refuses, with WD_ERR_ARG and the output untouched,
    every shape the stencil kernels do not support on this lattice (8x8x4x8:
    32 sites per plane of one parity, Lz = 4 so no z-slab order)."""
    import torch
    dims = (8, 8, 4, 8)
    V = li.volume(dims)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.random_su3_field(dims, 0.5, seed=61)), recon=12)
    inp = dev(li.gaussian_spinor(V // 2, seed=62, nrhs=2))
    out = torch.full_like(inp, 7 + 7j)
    bad = [(wd.WD_F16, (96, 1, 1, 0, 0)),     # threads not a multiple of 64
           (wd.WD_F16, (320, 1, 1, 0, 0)),    # more than 256 threads
           (wd.WD_F16, (128, 5, 1, 0, 0)),    # 5 RHS per lane
           (wd.WD_F16, (128, 1, 3, 0, 0)),    # 3 lanes per site
           (wd.WD_F16, (128, 1, 1, 18, 0)),   # no such tile order
           (wd.WD_F16, (128, 1, 1, 2, 0)),    # z-slab order with Lz = 4
           (wd.WD_F16, (128, 1, 1, 1, 1)),    # cap of 1 work-group per CU
           (wd.WD_F16, (128, 1, 1, 1, 9)),    # cap of 9
           (wd.WD_F16, (256, 1, 2, 8, 0)),    # LDS-staged with 2 lanes per site
           (wd.WD_F16, (128, 1, 1, 11, 0)),   # t-walking tile larger than a plane
           (wd.WD_F32, (64, 1, 1, 11, 0)),    # t-walking with FP32 spinors
           (wd.WD_F64, (128, 3, 1, 0, 0))]    # FP64 with 3 RHS per lane
    for code, shape in bad:
        with pytest.raises(wd.WDError) as e:
            wd.wd_dslash_shaped(lat.ctx, out, inp, wd.WD_ODD, 0, code, shape)
        assert e.value.status == wd.WD_ERR_ARG, (code, shape)
        assert bool((out == 7 + 7j).all()), (code, shape)
    lat.close()


def test_invalid_cache_lines_are_not_adopted(wd, tmp_path, monkeypatch):
    """Cache lines the lattice or the link format cannot run (non-temporal
    links with 18-real links, a z-slab order with Lz = 4, 96 threads) are
    ignored and those sweeps are timed afresh; the valid line is verified and
    adopted."""
    dims = (8, 8, 4, 8)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.random_su3_field(dims, 0.5, seed=63)), recon=12)
    key = "8 8 4 8 2 2 4"  # dims, nrhs 2, FP16 spinors, FP32 18-real links
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{key} 0 0 128 1 1 1 0 1.0 1\n"   # D_oe: lnt with 18-real links
                     f"{key} 0 1 128 1 1 2 0 1.0\n"     # xpay: z-slab order, Lz = 4
                     f"{key} 1 0 96 1 1 1 0 1.0\n"      # D_oe^dag: 96 threads
                     f"{key} 1 2 128 1 1 1 3 1.0\n")    # CG update: valid
    monkeypatch.setenv("WD_TUNE_CACHE", str(cache))
    rows = wd.wd_tune(lat.ctx, 2, wd.WD_F16 | wd.WD_LINKS_R18)
    assert [r["source"] for r in rows] == ["timed", "timed", "timed", "cache-verified"], rows
    assert all(r["rejected"] == 0 for r in rows) and rows[3]["occ"] == 3
    lat.close()
