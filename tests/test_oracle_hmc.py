"""Pins of the oracle's HMC pieces (Sec. 2 Hamiltonian and its three steps;
Sec. 3 gauge force, fermion force, gauge evolution): published Philox
known-answer vectors, finite differences of the actions against the forces,
gauge invariance, exactness of the start-of-trajectory fermion action,
equipartition, leapfrog reversibility and its dt^2 energy error."""
import os

import numpy as np
import pytest
import scipy.linalg

import lattice_inputs as li
from brute import dense_wilson, parity_sites, sites, lex, spin_colour_rows

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers(oracle):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_normals_moments(oracle):
    n = np.array([oracle.normal_pair(7, i, 3, 0x50, j) for i in range(20000) for j in range(2)])
    n = n.reshape(-1)
    assert abs(n.mean()) < 4 / np.sqrt(n.size)
    assert abs(n.var() - 1) < 5 * np.sqrt(2 / n.size)
    assert abs(np.mean(n ** 4) - 3) < 0.15


def test_momenta_hermitian_traceless_equipartition(oracle):
    dims = (4, 4, 4, 8)
    P = oracle.draw_momenta(dims, seed=5, traj=0)
    assert np.allclose(P, np.conj(np.swapaxes(P, -1, -2)))
    assert np.allclose(np.trace(P, axis1=-2, axis2=-1), 0)
    nl = P.shape[0] * 4
    K = oracle.kinetic(dims, P)
    # 1/2 tr p^2 = 1/2 sum of 8 unit normals per link: mean 4, variance 2 per link
    assert abs(K / nl - 4.0) < 5 * np.sqrt(2.0 / nl)
    # different trajectories draw different momenta; the same one repeats
    assert np.array_equal(P, oracle.draw_momenta(dims, seed=5, traj=0))
    assert not np.allclose(P, oracle.draw_momenta(dims, seed=5, traj=1))


def test_expi_matches_scipy(oracle):
    H = li.random_hermitian_traceless((5,), seed=9)
    for k in range(5):
        for a in (0.02, 0.7, 3.0):
            assert np.allclose(oracle.expi(H[k], a), scipy.linalg.expm(1j * a * H[k]), atol=1e-13)


def _gauge_transform(dims, U, g):
    c = sites(dims)
    out = np.empty_like(U)
    for x in range(len(c)):
        for mu in range(4):
            e = np.zeros(4, np.int64)
            e[mu] = 1
            out[x, mu] = g[x] @ U[x, mu] @ g[lex(dims, c[x] + e)].conj().T
    return out


def test_gauge_action_unit_and_invariance(oracle):
    dims = (4, 2, 4, 4)
    assert oracle.gauge_action(dims, li.unit_field(dims), 5.6) == 0.0
    assert np.abs(oracle.gauge_force(dims, li.unit_field(dims), 5.6)).max() < 1e-15
    U = li.random_su3_field(dims, 0.6, seed=2)
    g = li.random_su3(li.volume(dims), seed=3)
    Ug = _gauge_transform(dims, U, g)
    assert abs(oracle.plaquette(dims, U) - oracle.plaquette(dims, Ug)) < 1e-13
    # brute-force plaquette from the definition
    c = sites(dims)
    s = 0.0
    for x in range(len(c)):
        for mu in range(4):
            for nu in range(mu + 1, 4):
                em = np.zeros(4, np.int64); em[mu] = 1
                en = np.zeros(4, np.int64); en[nu] = 1
                P = (U[x, mu] @ U[lex(dims, c[x] + em), nu] @ U[lex(dims, c[x] + en), mu].conj().T
                     @ U[x, nu].conj().T)
                s += np.trace(P).real / 3
    assert abs(oracle.plaquette(dims, U) - s / (6 * len(c))) < 1e-13


def _move(U, X, t):
    """U_l -> exp(i t X_l) U_l on every link."""
    E = np.array([scipy.linalg.expm(1j * t * X[l]) for l in range(X.shape[0])])
    return np.einsum("lab,lbc->lac", E, U.reshape(-1, 3, 3)).reshape(U.shape)


def test_gauge_force_finite_difference(oracle):
    dims = (4, 2, 2, 4)
    beta = 5.6
    U = li.random_su3_field(dims, 0.5, seed=12)
    X = li.random_hermitian_traceless((li.volume(dims) * 4,), seed=13)
    F = oracle.gauge_force(dims, U, beta)
    assert np.allclose(F, np.conj(np.swapaxes(F, -1, -2)))
    assert np.allclose(np.trace(F, axis1=-2, axis2=-1), 0)
    pred = np.einsum("lab,lba->", X, F.reshape(-1, 3, 3)).real
    eps = 1e-4
    fd = (oracle.gauge_action(dims, _move(U, X, eps), beta) -
          oracle.gauge_action(dims, _move(U, X, -eps), beta)) / (2 * eps)
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))


def _dense_fermion_action(dims, U, kappa, phi, eo):
    M = dense_wilson(dims, U, kappa)
    if eo:
        ev, od = parity_sites(dims)
        re, ro = spin_colour_rows(ev), spin_colour_rows(od)
        M = np.eye(len(re)) - M[np.ix_(re, ro)] @ M[np.ix_(ro, re)]
    A = M.conj().T @ M
    return np.real(np.vdot(phi.reshape(-1), np.linalg.solve(A, phi.reshape(-1))))


@pytest.mark.parametrize("eo", [False, True])
def test_fermion_force_finite_difference(oracle, eo):
    dims = (2, 2, 2, 4)
    V = li.volume(dims)
    kappa = 0.12  # well inside the spectrum: the FD error is O(eps^2 |A^-1|^3)
    U = li.random_su3_field(dims, 0.5, seed=20)
    phi = li.gaussian_spinor(V // 2 if eo else V, seed=21)
    X = li.random_hermitian_traceless((V * 4,), seed=22)
    F, it = oracle.fermion_force(dims, U, kappa, phi, eo=eo, tol=1e-14)
    assert np.allclose(F, np.conj(np.swapaxes(F, -1, -2)))
    assert np.allclose(np.trace(F, axis1=-2, axis2=-1), 0)
    pred = np.einsum("lab,lba->", X, F.reshape(-1, 3, 3)).real
    eps = 1e-4
    fd = (_dense_fermion_action(dims, _move(U, X, eps), kappa, phi, eo) -
          _dense_fermion_action(dims, _move(U, X, -eps), kappa, phi, eo)) / (2 * eps)
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
    # the oracle's own action agrees with the dense solve
    s, _ = oracle.fermion_action(dims, U, kappa, phi, eo=eo, tol=1e-14)
    assert abs(s - _dense_fermion_action(dims, U, kappa, phi, eo)) < 1e-10 * abs(s)


def test_start_fermion_action_is_chi_squared(oracle):
    dims = (4, 4, 4, 4)
    U = li.random_su3_field(dims, 0.5, seed=30)
    U2, r = oracle.hmc_trajectory(dims, U, 5.6, 0.15, 0.2, 4, seed=77, traj=3, eo=True,
                                  tol_force=1e-10, tol_h=1e-13)
    chi = oracle.draw_chi(li.volume(dims) // 2, seed=77, traj=3)
    c2 = np.vdot(chi, chi).real
    assert abs(r["Sf_start"] - c2) < 1e-9 * c2


def test_leapfrog_reversible(oracle):
    dims = (2, 2, 4, 4)
    V = li.volume(dims)
    beta, kappa = 5.6, 0.12
    U = li.random_su3_field(dims, 0.5, seed=40)
    P = oracle.draw_momenta(dims, seed=41, traj=0)
    phi = li.gaussian_spinor(V // 2, seed=42)
    U1, P1, _ = oracle.leapfrog(dims, U, P, beta, kappa, phi, 0.5, 10, eo=True, tol=1e-14)
    U2, P2, _ = oracle.leapfrog(dims, U1, -P1, beta, kappa, phi, 0.5, 10, eo=True, tol=1e-14)
    assert np.abs(U2 - U).max() < 1e-10
    assert np.abs(P2 + P).max() < 1e-9


def test_energy_error_scales_as_dt_squared(oracle):
    dims = (4, 4, 4, 4)
    U = li.random_su3_field(dims, 0.4, seed=50)
    dh = []
    # kappa below the region where this rough field has near-zero modes of Mhat
    for n in (16, 32):
        _, r = oracle.hmc_trajectory(dims, U, 5.6, 0.12, 0.5, n, seed=51, traj=0, eo=True,
                                     tol_force=1e-13, tol_h=1e-13)
        dh.append(abs(r["dH"]))
    ratio = dh[0] / dh[1]
    assert 2.5 < ratio < 6.0, (dh, ratio)


def test_reject_restores_field(oracle):
    dims = (2, 2, 2, 2)
    U = li.random_su3_field(dims, 0.5, seed=60)
    # a huge step size gives a huge (or non-finite) dH: the proposal is
    # rejected and the field returned unchanged
    U2, r = oracle.hmc_trajectory(dims, U, 5.6, 0.12, 4.0, 2, seed=61, traj=0, eo=True)
    assert not np.isfinite(r["dH"]) or r["dH"] > 5
    assert not r["accepted"]
    assert np.array_equal(U2, U)


@pytest.mark.slow
def test_exp_minus_dh_averages_to_one(oracle):
    dims = (4, 4, 4, 4)
    U = li.random_su3_field(dims, 0.5, seed=70)
    vals = []
    for traj in range(120):
        U, r = oracle.hmc_trajectory(dims, U, 5.6, 0.12, 0.5, 8, seed=71, traj=traj, eo=True,
                                     tol_force=1e-10, tol_h=1e-12)
        if traj >= 10:
            vals.append(np.exp(-r["dH"]))
    vals = np.array(vals)
    m, se = vals.mean(), vals.std(ddof=1) / np.sqrt(len(vals))
    assert abs(m - 1) < max(3 * se, 0.02), (m, se)
