"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method itself (no Dirac operator, solver,
force or integrator): it only draws gauge fields, sources and test directions
from numpy's PCG64 generator.  Both the oracle side and the GPU side receive
exactly these arrays.

Recipes (the paper generates its fields in-program and prints none):
  gauge field   U = exp(i eps H) per link with H = sum_a xi_a lambda_a / 2,
                xi_a ~ N(0,1), then re-unitarised: rows 1 and 2 by Gram-Schmidt,
                row 3 = conj(row1 x row2) so that U is in SU(3) to round-off.
                Draw order: lex site, then mu, then a.
  source        complex Gaussian, Re and Im ~ N(0, 1/2) (density exp(-chi^dag chi)).
Layouts are the canonical complex128 ones: spinor [V][4][3], links [V][4][3][3].
"""
import numpy as np

__all__ = ["gell_mann", "random_su3_field", "unit_field", "gaussian_spinor",
           "random_su3", "random_hermitian_traceless", "volume", "config_seed"]


def volume(dims):
    return int(np.prod(dims))


def config_seed(index):
    """Seed of the numbered workload recipe (1000 + index)."""
    return 1000 + int(index)


def gell_mann():
    """The eight Gell-Mann matrices, shape [8][3][3]."""
    L = np.zeros((8, 3, 3), np.complex128)
    L[0][0, 1] = L[0][1, 0] = 1
    L[1][0, 1] = -1j
    L[1][1, 0] = 1j
    L[2][0, 0] = 1
    L[2][1, 1] = -1
    L[3][0, 2] = L[3][2, 0] = 1
    L[4][0, 2] = -1j
    L[4][2, 0] = 1j
    L[5][1, 2] = L[5][2, 1] = 1
    L[6][1, 2] = -1j
    L[6][2, 1] = 1j
    L[7][0, 0] = L[7][1, 1] = 1 / np.sqrt(3)
    L[7][2, 2] = -2 / np.sqrt(3)
    return L


def _reunitarise(M):
    """Rows 1-2 orthonormalised, row 3 = conj(row1 x row2); M has shape [..., 3, 3]."""
    r0 = M[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = M[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _expi_hermitian(H):
    """exp(i H) for a stack of Hermitian matrices by eigendecomposition."""
    w, v = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), np.conj(v))


def random_su3_field(dims, eps, seed):
    """Links [V][4][3][3] complex128 drawn by the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    V = volume(dims)
    xi = rng.standard_normal((V, 4, 8))
    H = np.einsum("sma,aij->smij", xi, gell_mann()) / 2.0
    U = _expi_hermitian(eps * H)
    return np.ascontiguousarray(_reunitarise(U))


def unit_field(dims):
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def gaussian_spinor(nsites, seed, nrhs=None):
    """Complex Gaussian spinor(s) [nsites][4][3] (or [nrhs][nsites][4][3])."""
    rng = np.random.default_rng(seed)
    shape = (nsites, 4, 3) if nrhs is None else (nrhs, nsites, 4, 3)
    s = np.sqrt(0.5)
    return np.ascontiguousarray(s * rng.standard_normal(shape) +
                                1j * s * rng.standard_normal(shape))


def random_su3(n, seed):
    """n Haar-distributed-ish SU(3) matrices (QR of a complex Gaussian, phases
    fixed, determinant divided out)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(_reunitarise(Q))


def random_hermitian_traceless(shape, seed):
    """Random traceless Hermitian 3x3 matrices sum_a xi_a lambda_a / sqrt(2)."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(tuple(shape) + (8,))
    return np.ascontiguousarray(np.einsum("...a,aij->...ij", xi, gell_mann()) / np.sqrt(2.0))
