"""Independent brute-force constructions used to pin the oracle.

Written from the definitions directly, sharing nothing with oracle/wdref.c:
the lattice is enumerated with numpy index arithmetic, the Wilson matrix is
assembled block by block as a dense array, and the gamma matrices are typed in
from the chiral (DeGrand-Rossi) basis.
"""
import itertools

import numpy as np

# chiral basis, gamma_1..gamma_4 for x, y, z, t
GAMMA = np.array([
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = np.diag([1, 1, -1, -1]).astype(np.complex128)


def sites(dims):
    """Coordinates of every site in lex order (x fastest) as an array [V][4]."""
    Lx, Ly, Lz, Lt = dims
    out = []
    for t, z, y, x in itertools.product(range(Lt), range(Lz), range(Ly), range(Lx)):
        out.append((x, y, z, t))
    return np.array(out, dtype=np.int64)


def lex(dims, c):
    Lx, Ly, Lz, Lt = dims
    c = np.asarray(c) % np.asarray(dims)
    return int(c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3])))


def dense_hopping(dims, U):
    """Dense H with (H psi)(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu).
    Index of (site, spin, colour) = site*12 + spin*3 + colour."""
    V = int(np.prod(dims))
    N = 12 * V
    H = np.zeros((N, N), np.complex128)
    I4 = np.eye(4)
    for xi, c in enumerate(sites(dims)):
        assert lex(dims, c) == xi
        for mu in range(4):
            e = np.zeros(4, np.int64)
            e[mu] = 1
            xf = lex(dims, c + e)
            xb = lex(dims, c - e)
            H[xi * 12:(xi + 1) * 12, xf * 12:(xf + 1) * 12] += np.kron(I4 - GAMMA[mu], U[xi, mu])
            H[xi * 12:(xi + 1) * 12, xb * 12:(xb + 1) * 12] += np.kron(I4 + GAMMA[mu],
                                                                      U[xb, mu].conj().T)
    return H


def dense_wilson(dims, U, kappa):
    H = dense_hopping(dims, U)
    return np.eye(H.shape[0]) - kappa * H


def parity_sites(dims):
    """Lex indices of the even and of the odd sites, each in cb (= lex>>1) order."""
    c = sites(dims)
    par = c.sum(axis=1) % 2
    V = len(c)
    ev = np.zeros(V // 2, np.int64)
    od = np.zeros(V // 2, np.int64)
    for l in range(V):
        (ev if par[l] == 0 else od)[l >> 1] = l
    return ev, od


def spin_colour_rows(site_list):
    return (np.asarray(site_list)[:, None] * 12 + np.arange(12)[None, :]).reshape(-1)


def free_spectrum(dims, kappa):
    """Eigenvalues of M^dag M for U = 1: (1 - 2k sum cos p)^2 + 4k^2 sum sin^2 p,
    p_mu = 2 pi n_mu / L_mu, each twelve-fold."""
    ps = [2 * np.pi * np.arange(L) / L for L in dims]
    vals = []
    for p in itertools.product(*ps):
        p = np.array(p)
        vals.append((1 - 2 * kappa * np.cos(p).sum()) ** 2 + 4 * kappa ** 2 * (np.sin(p) ** 2).sum())
    return np.sort(np.repeat(np.array(vals), 12))
