"""Host-side pieces of bench.py: the workload inputs follow the stated
recipe (a random SU(3) field, not the free field), the roofline arithmetic,
and the single-GPU guard."""
import subprocess
import sys
import os

import numpy as np
import pytest

import lattice_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_solve_workload_inputs_follow_the_recipe():
    import bench
    w = bench.WORKLOADS["c1_4c4"]
    U, B = bench.make_inputs(w)
    assert np.array_equal(U, li.random_su3_field(w["dims"], w["eps"], seed=li.config_seed(w["cfg"])))
    assert not np.allclose(U, li.unit_field(w["dims"]))
    assert B.shape == (w["nrhs"], li.volume(w["dims"]) // 2, 4, 3)


def test_kernel_roofline_arithmetic():
    import bench
    rep = {"a": (10, 20.0, 8e9, 1e7), "b": (10, 5.0, 1e9, 1e7)}
    dom, roof, sten = bench.kernel_roofline(rep, wall_s=0.05)
    assert dom["name"] == "a" and abs(dom["avg_us"] - 2000.0) < 1e-9
    assert abs(roof["achieved"] - 8e8 / 2e-3 / 1e9) < 1e-9
    assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-12
    assert abs(sten["share_of_step"] - 0.5) < 1e-12
    merged = bench.merge_reports([rep, {"a": (1, 1.0, 1.0, 1.0)}])
    assert merged["a"] == (11, 21.0, 8e9 + 1.0, 1e7 + 1.0)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_shape_table_lines_are_valid_launch_shapes():
    """The MI355X launch-shape table bench.py reuses: one line per sweep,
    dims nrhs sp lk dag epi block nr rl remap occ us [lnt], every field in
    range (tile orders 0-7 register-tiled, 8-10 LDS-staged, 11-13 t-walking;
    lnt = 1 only for FP16 or FP32 spinors over FP32 12- or 8-real links and
    FP64 spinors over FP64 12-real links, one lane per site, 1-2 RHS per
    lane, orders 0-7)."""
    import bench
    seen = set()
    for line in open(bench.SHAPE_TABLE):
        f = line.split()
        assert len(f) in (15, 16), line
        d = [int(x) for x in f[:14]]
        lx, ly, lz, lt, nrhs, sp, lk, dag, epi, block, nr, rl, remap, occ = d
        lnt = int(f[15]) if len(f) == 16 else 0
        assert all(L % 2 == 0 for L in (lx, ly, lz, lt)) and 1 <= nrhs <= 64
        assert sp in (0, 1, 2, 3) and lk in (0, 1, 2, 3, 4, 5) and dag in (0, 1) and epi in (0, 1, 2)
        assert block in (64, 128, 256) and nr in (1, 2, 3, 4) and rl in (1, 2, 4)
        assert 0 <= remap < 14 and (occ == 0 or 2 <= occ <= 8) and float(f[14]) > 0
        nt_fmt = (lk in (2, 5) and sp in (1, 2)) or (lk == 1 and sp == 0)
        assert lnt in (0, 1) and (lnt == 0 or (nt_fmt and rl == 1 and nr in (1, 2) and remap < 8)), line
        seen.add(tuple(d[:9]))
    # the four sweeps of the c3 workload's FP16 solve are all there
    assert all((32, 32, 32, 64, 12, 2, 2, dag, epi) in seen for dag, epi in ((0, 0), (0, 1), (1, 0), (1, 2)))


def test_shape_table_is_used_through_a_private_copy(monkeypatch):
    """bench.py points WD_TUNE_CACHE at a private copy of the table (the
    library appends to it), and leaves an explicit WD_TUNE_CACHE or
    --retune alone."""
    import os
    import sys
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    monkeypatch.delenv("WD_TUNE_CACHE", raising=False)
    bench.use_shape_table(bench.parse())
    dst = os.environ["WD_TUNE_CACHE"]
    assert dst != bench.SHAPE_TABLE and open(dst).read() == open(bench.SHAPE_TABLE).read()
    monkeypatch.setenv("WD_TUNE_CACHE", "/nonexistent/keep")
    bench.use_shape_table(bench.parse())
    assert os.environ["WD_TUNE_CACHE"] == "/nonexistent/keep"
    monkeypatch.delenv("WD_TUNE_CACHE")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--retune"])
    bench.use_shape_table(bench.parse())
    assert "WD_TUNE_CACHE" not in os.environ


def test_t_cut_share_needs_more_than_one_slab():
    """The one-GPU share of a t-cut lattice (slabs of 8 t-slices) is refused
    on the host for Lt <= 8, before any library call."""
    import bench
    with pytest.raises(ValueError):
        bench.shard_section(None, None, (4, 4, 4, 4))
    with pytest.raises(ValueError):
        bench.shard_section(None, None, (8, 8, 8, 8))


def test_line_contract_keys_and_cache_note():
    """The JSON line's fixed keys, the roofline entry's keys, and the
    cache-resident note only for launches that fit the last-level cache."""
    import argparse
    import bench
    args = argparse.Namespace(steps=20, warmup=1)
    rec = bench.base_record(args, 22.0, "solves/s", 545.0, "f16+norm/f32", {"workload": "w"})
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["vs_baseline"] is None and rec["config"]["workload"] == "w"
    big = {"k": (10, 7.4, 10 * 3.02e9, 10 * 12582912.0)}
    small = {"k": (10, 0.35, 10 * 1.34e8, 10 * 524288.0)}
    _, rb, _ = bench.kernel_roofline(big)
    _, rs, _ = bench.kernel_roofline(small)
    for r in (rb, rs):
        assert {"bound", "achieved", "peak", "unit", "frac", "traffic"} <= set(r)
    assert "note" not in rb and rs["note"].startswith("cache-resident")
