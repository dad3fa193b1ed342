"""Pins of the oracle's conjugate-gradient solver (eq. 3: the inverse applied by
CG) against a dense LU solve, the exact free-field solution in momentum space,
CG's monotone A-norm error and the even-odd reconstruction of a full solve."""
import numpy as np
import pytest

import lattice_inputs as li
from brute import dense_wilson, free_spectrum, parity_sites, spin_colour_rows, sites


def test_cg_full_matches_dense_lu(oracle):
    dims = (2, 2, 2, 2)
    V = 16
    U = li.random_su3_field(dims, 0.3, seed=1000)
    kappa = 0.15
    b = li.gaussian_spinor(V, seed=1)
    M = dense_wilson(dims, U, kappa)
    A = M.conj().T @ M
    x_ref = np.linalg.solve(A, b.reshape(-1))
    x, it, tr, ok = oracle.cg(dims, U, kappa, b, eo=False, tol=1e-10)
    assert ok and tr <= 1e-10
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x.reshape(-1) - x_ref) <= 1e-10 * cond * np.linalg.norm(x_ref)
    # the returned residual is the true one, recomputed from the dense matrix
    r = b.reshape(-1) - A @ x.reshape(-1)
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - tr) < 1e-14 * cond


def test_cg_eo_matches_dense_lu(oracle):
    dims = (2, 2, 2, 4)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=7)
    kappa = 0.155
    M = dense_wilson(dims, U, kappa)
    ev, od = parity_sites(dims)
    re, ro = spin_colour_rows(ev), spin_colour_rows(od)
    Mh = np.eye(len(re)) - (M[np.ix_(re, ro)] @ M[np.ix_(ro, re)])  # M_eo M_oe = k^2 D_eo D_oe
    A = Mh.conj().T @ Mh
    b = li.gaussian_spinor(V // 2, seed=8)
    x, it, tr, ok = oracle.cg(dims, U, kappa, b, eo=True, tol=1e-10)
    assert ok and tr <= 1e-10
    x_ref = np.linalg.solve(A, b.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - x_ref) <= 1e-10 * np.linalg.cond(A) * np.linalg.norm(x_ref)


def test_cg_free_field_fft_exact(oracle):
    """U = 1: M^dag M is diagonal in momentum space with eigenvalue lambda(p) on
    all 12 spin-colour components, so x = IFFT(FFT(b) / lambda)."""
    dims = (4, 4, 4, 8)
    V = li.volume(dims)
    kappa = 0.14
    U = li.unit_field(dims)
    b = li.gaussian_spinor(V, seed=99)
    Lx, Ly, Lz, Lt = dims
    bb = b.reshape(Lt, Lz, Ly, Lx, 12)
    bh = np.fft.fftn(bb, axes=(0, 1, 2, 3))
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(L) * 1.0 for L in (Lt, Lz, Ly, Lx)], indexing="ij")
    cos = sum(np.cos(k) for k in ks)
    sin2 = sum(np.sin(k) ** 2 for k in ks)
    lam = (1 - 2 * kappa * cos) ** 2 + 4 * kappa ** 2 * sin2
    x_ref = np.fft.ifftn(bh / lam[..., None], axes=(0, 1, 2, 3)).reshape(V, 4, 3)
    x, it, tr, ok = oracle.cg(dims, U, kappa, b, eo=False, tol=1e-12)
    assert ok
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    # a sanity bound from the spectrum: cond = lambda_max / lambda_min
    ev = free_spectrum(dims, kappa)
    assert it <= 10 * np.sqrt(ev[-1] / ev[0]) * 30


def test_cg_a_norm_error_decreases(oracle):
    dims = (2, 2, 2, 2)
    V = 16
    U = li.random_su3_field(dims, 0.4, seed=3)
    kappa = 0.15
    M = dense_wilson(dims, U, kappa)
    A = M.conj().T @ M
    b = li.gaussian_spinor(V, seed=4)
    x_ref = np.linalg.solve(A, b.reshape(-1))
    errs = []
    for k in range(1, 25):
        x, it, tr, ok = oracle.cg(dims, U, kappa, b, eo=False, tol=1e-30, maxiter=k)
        assert not ok and it == k
        e = x.reshape(-1) - x_ref
        errs.append(np.real(np.vdot(e, A @ e)))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_cg_zero_source_and_maxiter(oracle):
    dims = (2, 2, 2, 2)
    U = li.random_su3_field(dims, 0.3, seed=5)
    b = np.zeros((16, 4, 3), np.complex128)
    x, it, tr, ok = oracle.cg(dims, U, 0.15, b)
    assert ok and it == 0 and np.all(x == 0)


def test_eo_reconstruction_equals_full_solve(oracle):
    """Solving M x = b via Mhat: bhat_e = b_e + k D_eo b_o, Mhat x_e = bhat_e
    (normal equations with Mhat^dag), x_o = b_o + k D_oe x_e."""
    dims = (4, 2, 2, 4)
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.4, seed=9)
    kappa = 0.14
    b = li.gaussian_spinor(V, seed=10)
    ev, od = parity_sites(dims)
    be, bo = b[ev], b[od]
    bhat = be + kappa * oracle.hop_eo(dims, U, bo, 0)
    rhs = oracle.mhat(dims, U, kappa, bhat, dagger=True)
    xe, it, tr, ok = oracle.cg(dims, U, kappa, rhs, eo=True, tol=1e-13)
    assert ok
    xo = bo + kappa * oracle.hop_eo(dims, U, xe, 1)
    x = np.zeros_like(b)
    x[ev], x[od] = xe, xo
    M = dense_wilson(dims, U, kappa)
    x_ref = np.linalg.solve(M, b.reshape(-1)).reshape(V, 4, 3)
    assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
