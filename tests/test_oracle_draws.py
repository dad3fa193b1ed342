"""Pins of the oracle's two remaining random draws (Sec. 2: the pseudofermion
source chi is drawn from a Gaussian, and the trajectory is accepted or
rejected with a uniform number).

The pseudofermion weight exp(-phi^dag (M^dag M)^-1 phi) is reproduced by
phi = M^dag chi only if chi has density proportional to exp(-chi^dag chi):
each complex component then has independent real and imaginary parts of
variance 1/2, |chi_k|^2 is exponential with mean 1, and the 12 components of
one site give chi^dag chi ~ Gamma(12, 1).  The Metropolis test accepts with
probability min(1, exp(-dH)) only if u is uniform on (0, 1).  Every bound below
is a central-limit or Kolmogorov-Smirnov bound at several standard errors, so
that a wrong variance (a dropped sqrt(1/2)), a wrong scale of the 53-bit
uniform, or a shifted or folded distribution fails."""
import numpy as np
import pytest
import scipy.stats

NSITES = 20000           # 240000 complex components
SEED, TRAJ = 11, 4


@pytest.fixture(scope="module")
def chi(oracle):
    return oracle.draw_chi(NSITES, SEED, TRAJ)


def test_chi_component_variances(chi):
    re, im = chi.real.reshape(-1), chi.imag.reshape(-1)
    n = re.size
    for part in (re, im):
        # mean 0 and variance 1/2 per real component (standard errors
        # sqrt(1/2 / n) and sqrt(2 * (1/2)^2 / n))
        assert abs(part.mean()) < 5 * np.sqrt(0.5 / n)
        assert abs(part.var() - 0.5) < 5 * np.sqrt(2 * 0.25 / n)
        # Gaussian shape: fourth moment 3 sigma^4 = 3/4
        assert abs(np.mean(part ** 4) - 0.75) < 0.03
    # real and imaginary parts uncorrelated, components of a site uncorrelated
    assert abs(np.mean(re * im)) < 5 * 0.5 / np.sqrt(n)
    c = chi.reshape(NSITES, 12)
    assert abs(np.mean((c[:, 0] * np.conj(c[:, 1])).real)) < 5 * 0.5 / np.sqrt(NSITES)


def test_chi_modulus_is_unit_exponential(chi):
    a2 = (np.abs(chi) ** 2).reshape(-1)
    # E|chi_k|^2 = 1 (density exp(-|chi_k|^2)), variance 1
    assert abs(a2.mean() - 1.0) < 5 / np.sqrt(a2.size)
    assert scipy.stats.kstest(a2[:50000], "expon").pvalue > 1e-4


def test_chi_site_norm_is_gamma_12(chi):
    s = (np.abs(chi) ** 2).sum(axis=(1, 2))
    # <chi^dag chi> = 12 per site and the whole field's sum is 12 * nsites
    assert abs(s.sum() / (12 * NSITES) - 1.0) < 5 / np.sqrt(12 * NSITES)
    assert scipy.stats.kstest(s, scipy.stats.gamma(12).cdf).pvalue > 1e-4


def test_chi_draw_is_keyed(oracle, chi):
    again = oracle.draw_chi(64, SEED, TRAJ)
    assert np.array_equal(again, chi[:64])
    assert not np.allclose(oracle.draw_chi(64, SEED, TRAJ + 1), chi[:64])
    assert not np.allclose(oracle.draw_chi(64, SEED + 1, TRAJ), chi[:64])


def test_metropolis_uniform_range_and_moments(oracle):
    n = 100000
    u = np.array([oracle.uniform(SEED, i, TRAJ, 0x4D, 0) for i in range(n)])
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
    # the sample variance has standard error sqrt(Var((u - 1/2)^2) / n), Var = 1/180
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4
    # P(u < e^-dH) = e^-dH: the accept rate of a fixed dH is its Boltzmann factor
    for dH in (0.1, 0.7, 2.0):
        rate = np.mean(u < np.exp(-dH))
        p = np.exp(-dH)
        assert abs(rate - p) < 5 * np.sqrt(p * (1 - p) / n)


def test_metropolis_uniform_resolution(oracle):
    # 53 significant bits: distinct draws almost never collide, and the
    # values are not confined to a coarse grid
    u = np.array([oracle.uniform(3, i, 0, 0x4D, 0) for i in range(20000)])
    assert np.unique(u).size == u.size
    assert np.unique(np.round(u * 2 ** 40)).size > 19990
