"""Pins of the oracle's scatter denoising (Sec. 2.5, Eq. 5) and noise
assembly (Sec. 2.6) against what the paper and the mathematics fix: the
iteration's fixed point is the minimiser of the discretised energy of Eq. 2
(found here by scipy's L-BFGS-B on that energy), the decay factors of its
constant and checkerboard modes from linearising Eq. 5, the exact fixed point
of a flat image, and the calibration numbers the paper prints.  CPU only."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "noise_calibration.txt")


def noisy_smooth(seed, nv=10, nu=12, mean=120.0):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:nv, 0:nu]
    lam = mean * (1.0 + 0.4 * np.sin(x / 3.0) * np.cos(y / 4.0))
    return rng.poisson(lam).astype(np.float64)


def energy_and_grad(s, shat, beta):
    """E[S] = sum (S - Shat log S) + beta/2 sum over adjacent pixel pairs (S_a - S_b)^2."""
    dv = np.diff(s, axis=0)
    du = np.diff(s, axis=1)
    e = np.sum(s - shat * np.log(s)) + 0.5 * beta * (np.sum(dv * dv) + np.sum(du * du))
    g = 1.0 - shat / s
    g[:-1, :] -= beta * dv
    g[1:, :] += beta * dv
    g[:, :-1] -= beta * du
    g[:, 1:] += beta * du
    return e, g


@pytest.mark.parametrize("seed,beta", [(1, 0.05), (2, 0.2)])
def test_fixed_point_minimises_the_discretised_energy(oracle_lib, seed, beta):
    shat = noisy_smooth(seed)
    s = oracle_lib.denoise(shat, beta, iters=6000)
    res = minimize(lambda v: energy_and_grad(v.reshape(shat.shape), shat, beta), shat.ravel(), jac=True,
                   method="L-BFGS-B", bounds=[(1e-6, None)] * shat.size,
                   options=dict(ftol=1e-15, gtol=1e-11, maxiter=20000))
    ref = res.x.reshape(shat.shape)
    assert np.allclose(s, ref, rtol=2e-6, atol=0)
    # the result is smoother than the data (the point of Eq. 2)
    tv = lambda a: np.abs(np.diff(a, axis=0)).sum() + np.abs(np.diff(a, axis=1)).sum()
    assert tv(s) < 0.5 * tv(shat)


@pytest.mark.parametrize("omega", [0.8, 1.0, 0.5])
def test_constant_mode_decays_at_the_linearised_rate(oracle_lib, omega):
    """Shat = c everywhere, S = c (1 + eps): Eq. 5 gives S' - c = eps c (1 - omega / (4 beta c))."""
    c, beta, eps = 50.0, 0.03, 1e-7
    shat = np.full((6, 8), c)
    s1 = oracle_lib.denoise(shat, beta, iters=1, omega=omega, s0=shat * (1.0 + eps))
    expect = eps * c * (1.0 - omega / (4.0 * beta * c))
    assert np.allclose(s1 - c, expect, rtol=1e-5, atol=0)


def test_checkerboard_mode_decays_at_the_linearised_rate(oracle_lib):
    """Interior pixels: the four neighbours have the opposite sign, so
    S' - c = eps c (-1)^(i+j) (1 - 2 omega - omega / (4 beta c))."""
    c, beta, eps, omega = 80.0, 0.02, 1e-7, 0.8
    nv, nu = 7, 9
    sign = (-1.0) ** np.add.outer(np.arange(nv), np.arange(nu))
    shat = np.full((nv, nu), c)
    s1 = oracle_lib.denoise(shat, beta, iters=1, omega=omega, s0=c * (1.0 + eps * sign))
    expect = eps * c * sign * (1.0 - 2.0 * omega - omega / (4.0 * beta * c))
    assert np.allclose((s1 - c)[1:-1, 1:-1], expect[1:-1, 1:-1], rtol=1e-5, atol=0)


def test_flat_image_is_a_fixed_point_and_zeros_stay_finite(oracle_lib):
    shat = np.full((5, 7), 33.0)
    s = oracle_lib.denoise(shat, 0.1, iters=50)
    assert np.allclose(s, 33.0, rtol=1e-13)
    z = noisy_smooth(3)
    z[2:4, 3:6] = 0.0
    s = oracle_lib.denoise(z, 0.1, iters=200, s_floor=1e-3)
    assert np.isfinite(s).all() and (s >= 1e-3).all()
    # batched images are independent
    both = oracle_lib.denoise(np.stack([z, z[::-1]]), 0.1, iters=200, s_floor=1e-3)
    assert np.array_equal(both[0], s)
    assert np.array_equal(both[1], oracle_lib.denoise(z[::-1].copy(), 0.1, iters=200, s_floor=1e-3))


def test_noise_assembly(oracle_lib):
    rng = np.random.default_rng(4)
    p, s = rng.uniform(1, 2, 50), rng.uniform(0.1, 0.3, 50)
    phat, shat = p + rng.normal(0, 0.01, 50), s + rng.normal(0, 0.01, 50)
    n, img = oracle_lib.noise(phat, p, shat, s, 1.0)
    assert np.allclose(n, (phat - p) + (shat - s), rtol=0, atol=1e-15)
    assert np.allclose(img, phat + shat, rtol=1e-15)         # alpha = 1: the MC image itself
    n0, img0 = oracle_lib.noise(p, p, s, s, 0.37)
    assert np.all(n0 == 0.0) and np.allclose(img0, p + s)
    n2, _ = oracle_lib.noise(phat, p, shat, s, 0.25)
    assert np.allclose(n2, 0.25 * n, rtol=1e-15)


def test_noise_scale_reproduces_the_paper_calibration(oracle_lib):
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    # zeta = n_sim / k^2 as printed (to the printed digits)
    assert abs(vals["n_sim"] / vals["k"] ** 2 - vals["zeta"]) / vals["zeta"] < 1e-4
    for mas in (0.2, 1.0, 2.5):
        a = oracle_lib.noise_scale(vals["n_sim"], vals["zeta"], mas)
        assert abs(a - vals["k"] / np.sqrt(mas)) < 1e-4 * vals["k"] / np.sqrt(mas)
