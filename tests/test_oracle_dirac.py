"""Pins of the oracle's lattice, gamma matrices, Wilson operator and even-odd
blocks against things other than itself: brute-force enumeration, a dense
matrix assembled independently from the definition, the free-field closed
form, gamma5-hermiticity, gauge covariance and the Schur-complement identities.
"""
import numpy as np
import pytest

import lattice_inputs as li
from brute import (GAMMA, GAMMA5, dense_hopping, dense_wilson, free_spectrum, lex,
                   parity_sites, sites, spin_colour_rows)

SHAPES = [(2, 2, 2, 2), (4, 2, 2, 2), (2, 4, 2, 4), (2, 2, 6, 2)]


# --- lattice and index tables (Sec. 1 lattice; Sec. 3 neighbour routine) ---

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 8), (12, 12, 12, 24)])
def test_index_tables_brute_force(oracle, dims):
    nb, cb, par, eo = oracle.index_tables(dims)
    c = sites(dims)
    V = len(c)
    dims_a = np.array(dims)
    for mu in range(4):
        e = np.zeros(4, np.int64)
        e[mu] = 1
        fwd = (c + e) % dims_a
        bwd = (c - e) % dims_a
        lf = fwd[:, 0] + dims[0] * (fwd[:, 1] + dims[1] * (fwd[:, 2] + dims[2] * fwd[:, 3]))
        lb = bwd[:, 0] + dims[0] * (bwd[:, 1] + dims[1] * (bwd[:, 2] + dims[2] * bwd[:, 3]))
        assert np.array_equal(nb[:, 2 * mu], lf)
        assert np.array_equal(nb[:, 2 * mu + 1], lb)
        # involution: forward then backward returns to the site
        assert np.array_equal(nb[nb[:, 2 * mu], 2 * mu + 1], np.arange(V))
    assert np.array_equal(par, c.sum(axis=1) % 2)
    assert np.array_equal(cb, np.arange(V) >> 1)
    # nearest neighbours always have the other parity
    for k in range(8):
        assert np.all(par[nb[:, k]] != par)
    # eo tables: a bijection onto each parity, cb order
    ev, od = parity_sites(dims)
    assert np.array_equal(eo[0], ev) and np.array_equal(eo[1], od)
    assert len(np.unique(np.concatenate([eo[0], eo[1]]))) == V


def test_index_tables_reject_odd_dims(oracle):
    with pytest.raises(ValueError):
        oracle.index_tables((3, 4, 4, 4))
    with pytest.raises(ValueError):
        oracle.index_tables((4, 4, 0, 4))


# --- gamma matrices (Sec. 3: four constant 4x4 matrices) ---

def test_gamma_clifford_and_basis(oracle):
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        assert np.allclose(g[mu], GAMMA[mu])
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu))
        for s in (+1, -1):
            P = (np.eye(4) + s * g[mu]) / 2
            assert np.allclose(P @ P, P)
            assert np.linalg.matrix_rank(P) == 2
            assert np.count_nonzero(np.abs(np.eye(4) + s * g[mu]) > 0) == 8
    g5 = oracle.gamma(4)
    assert np.allclose(g5, GAMMA5)
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3])


# --- Wilson operator against an independently assembled dense matrix ---

@pytest.mark.parametrize("dims", SHAPES)
def test_hop_matches_dense(oracle, dims):
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.7, seed=11)
    psi = li.gaussian_spinor(V, seed=12)
    H = dense_hopping(dims, U)
    ref = (H @ psi.reshape(-1)).reshape(V, 4, 3)
    assert np.allclose(oracle.hop(dims, U, psi), ref, atol=1e-12, rtol=0)
    refd = (H.conj().T @ psi.reshape(-1)).reshape(V, 4, 3)
    assert np.allclose(oracle.hop(dims, U, psi, dagger=True), refd, atol=1e-12, rtol=0)
    kappa = 0.13
    M = np.eye(12 * V) - kappa * H
    assert np.allclose(oracle.wilson(dims, U, kappa, psi), (M @ psi.reshape(-1)).reshape(V, 4, 3))
    assert np.allclose(oracle.mdagm(dims, U, kappa, psi),
                       (M.conj().T @ M @ psi.reshape(-1)).reshape(V, 4, 3))


def test_dagger_is_conjugate_transpose_and_gamma5_hermitian(oracle):
    dims = (2, 2, 2, 2)
    V = 16
    U = li.random_su3_field(dims, 0.9, seed=3)
    kappa = 0.17
    N = 12 * V
    M = np.zeros((N, N), np.complex128)
    Md = np.zeros((N, N), np.complex128)
    for j in range(N):
        e = np.zeros(N, np.complex128)
        e[j] = 1
        M[:, j] = oracle.wilson(dims, U, kappa, e.reshape(V, 4, 3)).reshape(-1)
        Md[:, j] = oracle.wilson(dims, U, kappa, e.reshape(V, 4, 3), dagger=True).reshape(-1)
    assert np.allclose(Md, M.conj().T, atol=1e-13)
    G5 = np.kron(np.eye(V), np.kron(GAMMA5, np.eye(3)))
    assert np.allclose(G5 @ M @ G5, M.conj().T, atol=1e-13)


def test_gamma5_hermiticity_inner_products(oracle):
    dims = (4, 2, 6, 4)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=5)
    chi = li.gaussian_spinor(V, seed=6)
    psi = li.gaussian_spinor(V, seed=7)
    kappa = 0.15
    g5 = lambda v: np.einsum("st,xtc->xsc", GAMMA5, v)
    lhs = np.vdot(chi, oracle.wilson(dims, U, kappa, psi))
    rhs = np.vdot(g5(oracle.wilson(dims, U, kappa, g5(chi))), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    rhs2 = np.vdot(oracle.wilson(dims, U, kappa, chi, dagger=True), psi)
    assert abs(lhs - rhs2) < 1e-11 * abs(lhs)


# --- free field: momentum-space closed form ---

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 2, 6, 8)])
def test_free_field_plane_waves(oracle, dims):
    kappa = 0.15
    U = li.unit_field(dims)
    c = sites(dims)
    rng = np.random.default_rng(1)
    for trial in range(4):
        n = np.array([rng.integers(0, L) for L in dims])
        p = 2 * np.pi * n / np.array(dims)
        s = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (c @ p))
        psi = phase[:, None, None] * s[None]
        Mp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(
            GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
        ref = phase[:, None, None] * (Mp @ s)[None]
        assert np.allclose(oracle.wilson(dims, U, kappa, psi), ref, atol=1e-12)


def test_free_field_spectrum_dense(oracle):
    dims = (4, 2, 2, 4)
    V = li.volume(dims)
    kappa = 0.15
    U = li.unit_field(dims)
    N = 12 * V
    A = np.zeros((N, N), np.complex128)
    for j in range(N):
        e = np.zeros(N, np.complex128)
        e[j] = 1
        A[:, j] = oracle.mdagm(dims, U, kappa, e.reshape(V, 4, 3)).reshape(-1)
    ev = np.sort(np.linalg.eigvalsh((A + A.conj().T) / 2))
    assert np.allclose(ev, free_spectrum(dims, kappa), atol=1e-12)


def test_free_field_extremes_4444():
    # closed-form numbers at kappa = 0.15 on 4^4: lambda_min at p = 0, lambda_max at p = pi
    ev = free_spectrum((4, 4, 4, 4), 0.15)
    assert abs(ev[0] - 0.04) < 1e-14 and abs(ev[-1] - 4.84) < 1e-12


# --- gauge covariance ---

def test_gauge_covariance(oracle):
    dims = (4, 2, 4, 6)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.8, seed=21)
    psi = li.gaussian_spinor(V, seed=22)
    g = li.random_su3(V, seed=23)
    nb, _, _, _ = oracle.index_tables(dims)
    # brute-force neighbour lookup for the transform, independent of nb
    c = sites(dims)
    Ug = np.empty_like(U)
    for x in range(V):
        for mu in range(4):
            e = np.zeros(4, np.int64)
            e[mu] = 1
            xf = lex(dims, c[x] + e)
            Ug[x, mu] = g[x] @ U[x, mu] @ g[xf].conj().T
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    kappa = 0.14
    lhs = oracle.wilson(dims, Ug, kappa, gpsi)
    rhs = np.einsum("xab,xsb->xsa", g, oracle.wilson(dims, U, kappa, psi))
    assert np.allclose(lhs, rhs, atol=1e-12)


# --- even-odd blocks ---

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_even_odd_blocks_are_dense_blocks(oracle, dims):
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.6, seed=31)
    H = dense_hopping(dims, U)
    ev, od = parity_sites(dims)
    re, ro = spin_colour_rows(ev), spin_colour_rows(od)
    Deo = H[np.ix_(re, ro)]
    Doe = H[np.ix_(ro, re)]
    Hd = H.conj().T
    psi_o = li.gaussian_spinor(V // 2, seed=32)
    psi_e = li.gaussian_spinor(V // 2, seed=33)
    assert np.allclose(oracle.hop_eo(dims, U, psi_o, 0).reshape(-1), Deo @ psi_o.reshape(-1))
    assert np.allclose(oracle.hop_eo(dims, U, psi_e, 1).reshape(-1), Doe @ psi_e.reshape(-1))
    assert np.allclose(oracle.hop_eo(dims, U, psi_o, 0, dagger=True).reshape(-1),
                       Hd[np.ix_(re, ro)] @ psi_o.reshape(-1))
    # the diagonal parity blocks of H vanish: no even-even or odd-odd hopping
    assert np.abs(H[np.ix_(re, re)]).max() == 0 and np.abs(H[np.ix_(ro, ro)]).max() == 0
    kappa = 0.16
    Mh = np.eye(len(re)) - kappa ** 2 * Deo @ Doe
    assert np.allclose(oracle.mhat(dims, U, kappa, psi_e).reshape(-1), Mh @ psi_e.reshape(-1))
    assert np.allclose(oracle.mhat(dims, U, kappa, psi_e, dagger=True).reshape(-1),
                       Mh.conj().T @ psi_e.reshape(-1))
    assert np.allclose(oracle.mhatdag_mhat(dims, U, kappa, psi_e).reshape(-1),
                       Mh.conj().T @ Mh @ psi_e.reshape(-1))


def test_determinant_schur_identity(oracle):
    """det M = det Mhat because the odd-odd block of M is the identity."""
    dims = (2, 2, 2, 2)
    V = 16
    U = li.random_su3_field(dims, 0.9, seed=41)
    kappa = 0.2
    M = dense_wilson(dims, U, kappa)
    n = 12 * V // 2
    Mh = np.zeros((n, n), np.complex128)
    for j in range(n):
        e = np.zeros(n, np.complex128)
        e[j] = 1
        Mh[:, j] = oracle.mhat(dims, U, kappa, e.reshape(V // 2, 4, 3)).reshape(-1)
    s1, l1 = np.linalg.slogdet(M)
    s2, l2 = np.linalg.slogdet(Mh)
    assert abs(l1 - l2) < 1e-10 and abs(s1 - s2) < 1e-10
    G5 = np.kron(np.eye(V // 2), np.kron(GAMMA5, np.eye(3)))
    assert np.allclose(G5 @ Mh @ G5, Mh.conj().T, atol=1e-13)


def test_two_site_extent_forward_equals_backward(oracle):
    """On L_mu = 2 the sites x+mu and x-mu coincide; the two hopping terms then
    act on the same neighbour and add to 2 U psi (projectors sum to 2)."""
    dims = (2, 2, 2, 2)
    V = 16
    U = li.unit_field(dims)
    psi = li.gaussian_spinor(V, seed=51)
    nb, _, _, _ = oracle.index_tables(dims)
    ref = np.zeros_like(psi)
    for mu in range(4):
        ref += 2 * psi[nb[:, 2 * mu]]
    assert np.allclose(oracle.hop(dims, U, psi), ref)
