"""The expected values of the t-face test (tests/test_gpu_faces.py) are the
oracle's hopping block applied to psi masked to one boundary slice.  Here
that construction is pinned against the terms across a t-cut written out
from the definition of H in a dense matrix (tests/brute.py), for both
parities and H^dag: forward (1 -+ g_t) U_t(x) psi(x + t) on slice Lt-1,
backward (1 +- g_t) U_t(x - t)^dag psi(x - t) on slice 0."""
import numpy as np
import pytest

import lattice_inputs as li
from brute import GAMMA, lex, parity_sites, sites, spin_colour_rows

DIMS = [(2, 2, 2, 4), (4, 2, 2, 6)]


def dense_cut_terms(dims, U, dagger):
    V = int(np.prod(dims))
    Lt = dims[3]
    C = np.zeros((12 * V, 12 * V), np.complex128)
    I4 = np.eye(4)
    s = -1 if not dagger else 1          # forward projector 1 + s g_t
    e = np.array([0, 0, 0, 1])
    for xi, c in enumerate(sites(dims)):
        if c[3] == Lt - 1:
            y = lex(dims, c + e)
            C[xi * 12:(xi + 1) * 12, y * 12:(y + 1) * 12] += np.kron(I4 + s * GAMMA[3], U[xi, 3])
        if c[3] == 0:
            y = lex(dims, c - e)
            C[xi * 12:(xi + 1) * 12, y * 12:(y + 1) * 12] += np.kron(I4 - s * GAMMA[3], U[y, 3].conj().T)
    return C


@pytest.mark.parametrize("dims", DIMS)
def test_masked_hop_is_the_cut_terms(oracle, dims):
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=65)
    ev, od = parity_sites(dims)
    tslice = np.arange(V // 2) // (dims[0] * dims[1] * dims[2] // 2)
    assert all(sites(dims)[ev][k][3] == tslice[k] for k in range(V // 2))
    Lt = dims[3]
    for dag in (False, True):
        C = dense_cut_terms(dims, U, dag)
        for out_par in (0, 1):
            rows = spin_colour_rows(ev if out_par == 0 else od)
            cols = spin_colour_rows(od if out_par == 0 else ev)
            psi = li.gaussian_spinor(V // 2, seed=66 + out_par)
            ref = (C[np.ix_(rows, cols)] @ psi.reshape(-1)).reshape(V // 2, 4, 3)
            pf = np.where((tslice == 0)[:, None, None], psi, 0)
            pb = np.where((tslice == Lt - 1)[:, None, None], psi, 0)
            hf = oracle.hop_eo(dims, U, pf, out_par, dagger=dag)
            hb = oracle.hop_eo(dims, U, pb, out_par, dagger=dag)
            got = np.zeros_like(psi)
            got[tslice == Lt - 1] = hf[tslice == Lt - 1]
            got[tslice == 0] = hb[tslice == 0]
            assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (dag, out_par)
