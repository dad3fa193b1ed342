"""Pins of the oracle's end-of-trajectory measurements (the Polyakov loop and
the point-source pion correlator; Sec. 3 measures on each configuration
without naming the observables).

* Free field (U = 1): the propagator M^-1 delta is (1/V) sum_p e^{ip(x-x0)}
  M(p)^-1 with M(p) = 1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu
  sin p_mu, evaluated here by FFT -- a momentum-space computation sharing
  nothing with the oracle's position-space CG.  It fixes every entry of the
  propagator and hence the correlator.
* Gauge invariance of the correlator under a random SU(3) transform.
* Polyakov loop: closed form for constant diagonal time links, the centre
  phase exp(2 pi i / 3) when one time slice is multiplied by it, gauge
  invariance for non-commuting links (which fixes the path order).
"""
import numpy as np
import pytest

import lattice_inputs as li
from brute import GAMMA


def free_propagator_fft(dims, kappa, src):
    """S[x][s'][s] = (M^-1 delta_src)(x) for U = 1 by the momentum sum."""
    Lx, Ly, Lz, Lt = dims
    P = np.meshgrid(*[2 * np.pi * np.arange(L) / L for L in dims], indexing="ij")
    cos = sum(np.cos(p) for p in P)
    Minv = np.zeros(tuple(dims) + (4, 4), np.complex128)
    I4 = np.eye(4)
    M = (1 - 2 * kappa * cos)[..., None, None] * I4
    for mu in range(4):
        M = M + 2j * kappa * np.sin(P[mu])[..., None, None] * GAMMA[mu]
    Minv = np.linalg.inv(M)
    # S(x) = (1/V) sum_p e^{i p (x - x0)} Minv(p)  -> inverse FFT along each axis
    S = np.fft.ifftn(Minv, axes=(0, 1, 2, 3))          # (1/V) sum_p e^{ipx} Minv(p)
    S = np.roll(S, shift=tuple(src), axis=(0, 1, 2, 3))  # x -> x - x0
    # to lex order [t][z][y][x] -> lex = x + Lx(y + Ly(z + Lz t))
    S = np.transpose(S, (3, 2, 1, 0, 4, 5)).reshape(-1, 4, 4)
    return S


@pytest.mark.parametrize("dims,src", [((4, 4, 4, 4), (0, 0, 0, 0)), ((4, 4, 4, 6), (1, 2, 3, 5)),
                                      ((2, 4, 2, 4), (1, 0, 0, 2))])
def test_free_propagator_and_correlator_match_momentum_space(oracle, dims, src):
    kappa = 0.11
    psi, st, _ = oracle.point_propagator(dims, li.unit_field(dims), kappa, src, tol=1e-13)
    assert st == 0
    S = free_propagator_fft(dims, kappa, src)
    V = li.volume(dims)
    ref = np.zeros((12, V, 4, 3), np.complex128)
    for s in range(4):
        for c in range(3):
            ref[3 * s + c, :, :, c] = S[:, :, s]
    assert np.abs(psi - ref).max() <= 1e-10 * np.abs(ref).max()
    corr = oracle.pion_correlator(dims, psi, src)
    v3 = dims[0] * dims[1] * dims[2]
    Sx = S.reshape(dims[3], v3, 4, 4)
    ref_c = np.array([3 * np.sum(np.abs(Sx[(src[3] + dt) % dims[3]]) ** 2) for dt in range(dims[3])])
    assert np.allclose(corr, ref_c, rtol=1e-10, atol=0)
    # free field: time-reflection symmetric about the source
    assert np.allclose(corr[1:], corr[1:][::-1], rtol=1e-9)


def _gauge_transform(dims, U, g):
    Up = U.copy()
    V = li.volume(dims)
    Lx, Ly, Lz, Lt = dims
    for x in range(V):
        c = [x % Lx, (x // Lx) % Ly, (x // (Lx * Ly)) % Lz, x // (Lx * Ly * Lz)]
        for mu in range(4):
            cc = list(c)
            cc[mu] = (cc[mu] + 1) % dims[mu]
            xp = cc[0] + Lx * (cc[1] + Ly * (cc[2] + Lz * cc[3]))
            Up[x, mu] = g[x] @ U[x, mu] @ g[xp].conj().T
    return Up


def test_correlator_is_gauge_invariant(oracle):
    dims, src, kappa = (4, 4, 4, 4), (1, 0, 3, 2), 0.12
    U = li.random_su3_field(dims, 0.4, seed=81)
    g = li.random_su3(li.volume(dims), seed=82)
    Ug = _gauge_transform(dims, U, g)
    c0 = oracle.pion_correlator(dims, oracle.point_propagator(dims, U, kappa, src, tol=1e-13)[0], src)
    c1 = oracle.pion_correlator(dims, oracle.point_propagator(dims, Ug, kappa, src, tol=1e-13)[0], src)
    assert np.allclose(c0, c1, rtol=1e-9)
    # and the propagator solves M psi = delta by the oracle's operator
    psi = oracle.point_propagator(dims, U, kappa, src, tol=1e-13)[0]
    s0 = src[0] + 4 * (src[1] + 4 * (src[2] + 4 * src[3]))
    for j in (0, 7, 11):
        b = np.zeros((li.volume(dims), 4, 3), np.complex128)
        b[s0, j // 3, j % 3] = 1
        assert np.linalg.norm(oracle.wilson(dims, U, kappa, psi[j]) - b) <= 1e-10


def test_polyakov_closed_forms_and_symmetries(oracle):
    dims = (4, 2, 2, 6)
    V, Lt = li.volume(dims), dims[3]
    assert oracle.polyakov(dims, li.unit_field(dims)) == pytest.approx(1.0, abs=1e-15)
    # constant diagonal time links: P = (1/3) sum_k exp(i Lt th_k)
    th = np.array([0.3, -0.1, -0.2])
    U = li.unit_field(dims)
    U[:, 3] = np.diag(np.exp(1j * th))
    ref = np.mean(np.exp(1j * Lt * th))
    assert abs(oracle.polyakov(dims, U) - ref) <= 1e-14
    # centre transformation of one time slice multiplies P by omega
    U = li.random_su3_field(dims, 0.5, seed=91)
    p0 = oracle.polyakov(dims, U)
    v3 = V // Lt
    Uc = U.copy()
    Uc[2 * v3:3 * v3, 3] *= np.exp(2j * np.pi / 3)
    assert abs(oracle.polyakov(dims, Uc) - np.exp(2j * np.pi / 3) * p0) <= 1e-13
    # gauge invariance with non-commuting links fixes the path order
    g = li.random_su3(V, seed=92)
    assert abs(oracle.polyakov(dims, _gauge_transform(dims, U, g)) - p0) <= 1e-13
    # the reversed product is not invariant: the order matters on this field
    Ut = U[:, 3].reshape(Lt, v3, 3, 3)
    rev = np.mean([np.trace(np.linalg.multi_dot(list(Ut[::-1, s]))) / 3 for s in range(v3)])
    assert abs(rev - p0) > 1e-3
