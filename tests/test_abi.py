"""The C-ABI library loads and exports every function include/wd.h declares
(no compute calls: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("wd_", "hmc_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("wd_create", "wd_destroy", "wd_gauge_load", "wd_dslash", "wd_mdagm",
                     "wd_cg_solve", "wd_index_tables", "wd_debug_device_tables"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1207_2223_amd import wd
    L = ctypes.CDLL(wd.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1207_2223_amd import wd
    missing = [n for n in declared_functions() if not callable(getattr(wd, n, None))]
    assert not missing, missing


def test_host_index_tables_match_oracle(oracle):
    from paper_1207_2223_amd import wd
    for dims in [(2, 2, 2, 2), (4, 2, 6, 8), (6, 4, 4, 6)]:
        nb, cb, par = wd.wd_index_tables(dims)
        onb, ocb, opar, _ = oracle.index_tables(dims)
        assert (nb == onb).all() and (cb == ocb).all() and (par == opar).all()


def test_bad_dims_rejected_without_gpu():
    from paper_1207_2223_amd import wd
    with pytest.raises(wd.WDError) as e:
        wd.wd_index_tables((3, 4, 4, 4))
    assert e.value.status == wd.WD_ERR_DIMS
    assert wd.wd_bytes_required((3, 4, 4, 4), 1) == 0
    assert wd.wd_bytes_required((16, 16, 16, 32), 1) > 0
    # one parity's 16-byte chunk array must stay addressable with 32-bit
    # byte offsets: 152^4 (Vh = 266887168) fits, 154^4 (Vh = 281224328) not
    assert wd.wd_bytes_required((152, 152, 152, 152), 1) > 0
    assert wd.wd_bytes_required((154, 154, 154, 154), 1) == 0


def test_solver_defaults():
    from paper_1207_2223_amd import wd
    p = wd.wd_solver_defaults()
    assert p.tol == 1e-10 and p.eo == 1 and p.prec_sloppy == wd.WD_F64
