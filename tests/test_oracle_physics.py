"""Pins of the oracle's interaction physics (Sec. 2.4: Compton and Rayleigh
angles from their differential cross sections) and of the synthetic cross
sections it consumes.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_1204_6367_amd import workloads as W

ME = 510.99895
HC = 12.398419843


def kn_dsigma_dcos(c, e_kev):
    """Klein-Nishina d(sigma)/d(cos theta) per electron in units of pi r_e^2."""
    k = e_kev / ME
    P = 1.0 / (1.0 + k * (1.0 - c))
    return P * P * (P + 1.0 / P - (1.0 - c * c))


def _chi2_against(samples, density, edges):
    counts, _ = np.histogram(samples, edges)
    probs = np.array([integrate.quad(density, a, b, epsabs=0, epsrel=1e-10)[0]
                      for a, b in zip(edges[:-1], edges[1:])])
    probs /= probs.sum()
    exp = probs * len(samples)
    keep = exp > 20
    return stats.chisquare(counts[keep], exp[keep] * counts[keep].sum() / exp[keep].sum()).pvalue


@pytest.mark.parametrize("e_kev", [20.0, 60.0, 150.0])
def test_compton_angle_follows_klein_nishina(oracle_lib, e_kev):
    cost, tau = oracle_lib.sample_compton(e_kev, seed=11, n=400000)
    assert np.all((cost >= -1.0 - 1e-12) & (cost <= 1.0 + 1e-12))
    k = e_kev / ME
    # energy-angle relation of Compton kinematics
    assert np.allclose(tau, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12, atol=0)
    edges = np.linspace(-1, 1, 41)
    assert _chi2_against(cost, lambda c: kn_dsigma_dcos(c, e_kev), edges) > 1e-4


def test_compton_thomson_limit(oracle_lib):
    """kappa -> 0: d(sigma)/d(cos) -> (1 + cos^2) (Thomson)."""
    cost, tau = oracle_lib.sample_compton(0.01, seed=12, n=300000)
    assert np.allclose(tau, 1.0, atol=1e-4)
    edges = np.linspace(-1, 1, 31)
    assert _chi2_against(cost, lambda c: 1.0 + c * c, edges) > 1e-4
    # mean cos is 0 and <cos^2> = 2/5 for the Thomson density
    assert abs(cost.mean()) < 0.005
    assert abs((cost**2).mean() - 0.4) < 0.005


def test_compton_rejects_wrong_density(oracle_lib):
    """The chi-square machinery has power: the 60 keV sample fails the Thomson law."""
    cost, _ = oracle_lib.sample_compton(60.0, seed=13, n=400000)
    assert _chi2_against(cost, lambda c: 1.0 + c * c, np.linspace(-1, 1, 41)) < 1e-6


def rayleigh_density(c, e_kev, x0):
    lam = HC / e_kev
    x = np.sqrt(np.maximum(0.0, (1.0 - c) / 2.0)) / lam
    return (1.0 + c * c) * np.exp(-2.0 * x / x0)


@pytest.mark.parametrize("e_kev", [2.0, 4.0, 30.0, 100.0])
def test_rayleigh_angle_follows_form_factor(oracle_lib, e_kev):
    x0 = W.RAYLEIGH_X0
    cost = oracle_lib.sample_rayleigh(e_kev, x0, seed=21, n=300000)
    assert np.all((cost >= -1.0) & (cost <= 1.0))
    # forward-peaked at high energy: bins dense near cos = 1
    edges = np.unique(np.concatenate([np.linspace(-1, 0.9, 20), 1.0 - np.geomspace(1e-4, 0.1, 20), [1.0]]))
    assert _chi2_against(cost, lambda c: rayleigh_density(c, e_kev, x0), edges) > 1e-4


def test_rayleigh_total_cross_section_matches_density():
    """The tabulated Rayleigh coefficient is the integral of the same density the
    sampler draws from: sigma/Z^2 = (r_e^2/2) 2 pi int (1+c^2) F^2/Z^2 dc."""
    for e in [5.0, 60.0, 140.0]:
        num = integrate.quad(lambda c: rayleigh_density(c, e, W.RAYLEIGH_X0), -1, 1,
                             epsrel=1e-10, points=[1 - 1e-3, 1 - 1e-2])[0]
        sigma = math.pi * W.R_ELECTRON_CM**2 * num
        tab = W.rayleigh_sigma_cm2_per_z(np.array([e]))[0]
        assert abs(tab - sigma) / sigma < 1e-6


def test_klein_nishina_total():
    """sigma_KN(60 keV)/sigma_Thomson = 0.8202 (textbook); and the total equals
    the integral of the differential cross section the sampler uses."""
    sT = 8.0 / 3.0 * math.pi * W.R_ELECTRON_CM**2
    assert abs(W.klein_nishina_sigma_cm2(np.array([60.0]))[0] / sT - 0.8202) < 5e-4
    for e in [10.0, 60.0, 150.0]:
        num = math.pi * W.R_ELECTRON_CM**2 * integrate.quad(lambda c: kn_dsigma_dcos(c, e), -1, 1)[0]
        assert abs(W.klein_nishina_sigma_cm2(np.array([e]))[0] - num) / num < 1e-10
    # low-energy limit: sigma/sigma_T = 1 - 2k + 26k^2/5 - ... (Thomson as k -> 0)
    k = 1.0 / ME
    assert abs(W.klein_nishina_sigma_cm2(np.array([1.0]))[0] / sT - (1 - 2 * k + 5.2 * k * k)) < 1e-6


def test_water_attenuation_levels():
    """Synthetic water: mu/rho(60 keV) ~ 0.2075 cm^2/g; photoelectric equals
    Compton near 27 keV (the design values of the synthetic tables)."""
    mu = W.mass_attenuation(W.MATERIALS["water"], np.array([60.0, 27.2]))
    assert abs(mu[0].sum() - 0.2075) < 5e-4
    assert abs(mu[1, 2] / mu[1, 1] - 1.0) < 0.01


def test_rotation_invariants(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(300):
        d = rng.standard_normal(3)
        if rng.random() < 0.2:                        # exercise the near-axis branch
            d = np.array([1e-4 * rng.standard_normal(), 1e-4 * rng.standard_normal(), np.sign(rng.standard_normal())])
        d /= np.linalg.norm(d)
        c = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * math.pi)
        o = oracle_lib.rotate(d, c, ph)
        assert abs(np.linalg.norm(o) - 1.0) < 1e-12
        assert abs(o @ d - c) < 1e-9


def test_rotation_azimuth_is_uniform(oracle_lib):
    """Over a uniform azimuth the new direction averages to cos(theta) d and its
    transverse part is isotropic in the plane normal to d."""
    d = np.array([0.3, -0.5, 0.8])
    d /= np.linalg.norm(d)
    c = 0.4
    phs = np.linspace(0, 2 * math.pi, 3600, endpoint=False)
    o = np.array([oracle_lib.rotate(d, c, p) for p in phs])
    assert np.allclose(o.mean(0), c * d, atol=1e-9)
    t = o - c * d[None, :]
    cov = t.T @ t / len(phs)
    s2 = 1 - c * c
    proj = np.eye(3) - np.outer(d, d)
    assert np.allclose(cov, 0.5 * s2 * proj, atol=1e-9)
    # successive azimuths turn the same way about d (a consistent frame)
    cr = np.cross(t[:-1], t[1:]) @ d
    assert np.all(cr > 0) or np.all(cr < 0)
