"""The allocation-free normal operator (wd_mdagm_noalloc, for callers that
cannot allocate) against wd_mdagm on the same inputs: the same kernels on a
fixed device array, so the same bits.  Two calls in a row, the second on a
smaller lattice (the array keeps the first call's contents), for the
even-odd and the full operator; a lattice beyond the array is refused."""
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


@pytest.mark.parametrize("eo", [1, 0])
def test_noalloc_equals_mdagm_two_calls_second_smaller(wd, oracle, eo):
    big = (16, 16, 16, 32) if eo else (12, 12, 12, 24)
    small = (6, 4, 4, 6)
    for k, dims in enumerate((big, small)):
        V = li.volume(dims)
        U = li.random_su3_field(dims, 0.5, seed=1300 + k)
        lat = wd.Lattice(dims)
        lat.gauge_load(dev(U), recon=12)
        psi = li.gaussian_spinor(V // 2 if eo else V, seed=1310 + k)
        kappa = 0.153 + 0.002 * k
        ref = empty_like_dev(psi)
        out = empty_like_dev(psi)
        lat.mdagm(ref, dev(psi), kappa, eo=eo)
        wd.wd_mdagm_noalloc(lat.ctx, out, dev(psi), kappa, eo)
        a, b = host(out), host(ref)
        note(f"noalloc eo {eo} {dims}: bitwise equal {np.array_equal(a.view(np.uint64), b.view(np.uint64))}")
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        if k == 1:  # and the small one against the oracle, to the FP64 bar
            o = oracle.mhatdag_mhat(dims, U, kappa, psi) if eo else oracle.mdagm(dims, U, kappa, psi)
            assert rel_err(a, o) <= 1e-12
        lat.close()


def test_noalloc_refuses_a_lattice_beyond_its_array(wd):
    dims = (16, 16, 16, 32)  # the full operator needs 6 x 12.7 MB > 64 MiB
    V = li.volume(dims)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.unit_field(dims)), recon=12)
    psi = dev(li.gaussian_spinor(V, seed=3))
    out = empty_like_dev(psi)
    with pytest.raises(wd.WDError) as e:
        wd.wd_mdagm_noalloc(lat.ctx, out, psi, 0.15, 0)
    assert e.value.status == wd.WD_ERR_ARG and "scratch" in str(e.value)
    lat.close()
