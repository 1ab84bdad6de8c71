"""Pins of the oracle's ray-tracing primary (Sec. 2.3, Eq. 1) against what the
paper and the mathematics fix: Beer-Lambert in closed form on a homogeneous
box, convergence to the exact line integral of the trilinearly interpolated
attenuation field (computed here by Gauss-Legendre quadrature between the
field's breakpoints, through scipy's linear grid interpolator), the
voxel-constant field with interpolation off, agreement with the independent
exact-integral primary of the MC check, symmetry, and where the shadow falls.
CPU only."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from paper_1204_6367_amd import workloads as W

from test_oracle_transport import geo_frame, make

GRID = W.EnergyGrid()


def pixel_rays(g, pix):
    """Source point and unit directions towards the centres of pixels `pix`."""
    S, P, n, eu, ev = geo_frame(g.phi_rad, g.theta_rad, g.sad_mm, g.aid_mm)
    iu, iv = np.asarray(pix) % g.nu, np.asarray(pix) // g.nu
    uc = (iu + 0.5 - 0.5 * g.nu) * g.du_mm
    vc = (iv + 0.5 - 0.5 * g.nv) * g.dv_mm
    D = P[None] + uc[:, None] * eu[None] + vc[:, None] * ev[None]
    d = D - S[None]
    ln = np.linalg.norm(d, axis=1)
    return S, d / ln[:, None], ln


def chord(S, d, half):
    """[t_in, t_out] of the ray S + t d in the box |x_a| <= half_a (slab method)."""
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if abs(S[a]) > half[a]:
                return None
            continue
        ta, tb = sorted(((-half[a] - S[a]) / d[a], (half[a] - S[a]) / d[a]))
        t0, t1 = max(t0, ta), min(t1, tb)
    return (t0, t1) if t0 < t1 else None


def mu_total(names, e):
    """Total mass attenuation [n_mat] at energy e, linear in E between grid points."""
    tab = W.cross_section_table(names, GRID).astype(np.float64).sum(-1)
    eg = GRID.e0_kev + GRID.de_kev * np.arange(GRID.n_e)
    return np.array([np.interp(e, eg, tab[m]) for m in range(len(names))])


def mu_field(ph, e, interp):
    """The attenuation field mu(x, E) (1/cm) as a callable on points [k][3] (x, y, z)."""
    nz, ny, nx = ph.shape
    dx, dy, dz = ph.spacing_mm
    vox = ph.density.astype(np.float64) * mu_total(ph.materials, e)[ph.material]
    if not interp:
        def f(x):
            i = [np.clip(np.floor((x[:, a] + 0.5 * n * s) / s).astype(int), 0, n - 1)
                 for a, (n, s) in enumerate(((nx, dx), (ny, dy), (nz, dz)))]
            return vox[i[2], i[1], i[0]]
        return f
    # centres plus the box faces, with the edge values repeated: linear
    # interpolation on that grid is trilinear with clamping at the edges
    axes = []
    for n, s in ((nz, dz), (ny, dy), (nx, dx)):
        c = (np.arange(n) + 0.5 - 0.5 * n) * s
        axes.append(np.concatenate([[-0.5 * n * s], c, [0.5 * n * s]]))
    it = RegularGridInterpolator(axes, np.pad(vox, 1, mode="edge"), method="linear")
    return lambda x: it(x[:, ::-1])


def exact_line_integral(ph, f, S, d, tlim, interp):
    """Integral of f along S + t d over [t_in, t_out] (mm * 1/cm): Gauss-Legendre
    (4 nodes, exact for the cubic pieces) between the planes where the
    field's pieces change (voxel faces, and centres when interpolating)."""
    nz, ny, nx = ph.shape
    dx, dy, dz = ph.spacing_mm
    t0, t1 = tlim
    br = [t0, t1]
    for a, (n, s) in enumerate(((nx, dx), (ny, dy), (nz, dz))):
        if d[a] == 0.0:
            continue
        planes = (np.arange(2 * n + 1) * 0.5 - 0.5 * n) * s if interp else (np.arange(n + 1) - 0.5 * n) * s
        t = (planes - S[a]) / d[a]
        br.extend(t[(t > t0) & (t < t1)])
    br = np.unique(np.array(br))
    gx, gw = np.polynomial.legendre.leggauss(4)
    a, b = br[:-1], br[1:]
    tt = 0.5 * (a + b)[:, None] + 0.5 * (b - a)[:, None] * gx[None]
    vals = f((S[None, None] + tt[..., None] * d[None, None]).reshape(-1, 3)).reshape(tt.shape)
    return float((0.5 * (b - a) * (vals * gw[None]).sum(1)).sum())


def random_phantom(seed, shape=(6, 5, 7), spacing=(4.0, 3.0, 5.0), names=("water", "bone", "lung")):
    rng = np.random.default_rng(seed)
    m = rng.integers(0, len(names), shape).astype(np.uint8)
    dens = rng.uniform(0.3, 2.0, shape).astype(np.float32)
    return W.Phantom(dens, m, spacing, list(names))


def test_homogeneous_box_is_beer_lambert_in_closed_form(oracle_lib):
    """Constant density, one material: the interpolated field is constant, the
    interval lengths add up to the chord, so P(u) = w(u) sum_k phi_k r(E_k)
    exp(-rho mu(E_k) chord) exactly, for any dl, with or without interpolation.
    Channel energies off the table grid, a non-trivial response and
    unnormalised spectrum and fluence weights."""
    ph = W.box_phantom((10, 12, 14), (2.0, 2.5, 3.0), "water", density=0.8)
    g = W.Geometry(phi_rad=0.4, theta_rad=0.1, nu=24, nv=16, du_mm=6.0, dv_mm=6.0)
    rng = np.random.default_rng(3)
    flu = rng.uniform(0.5, 2.0, (g.nv, g.nu)).astype(np.float32)
    flu64 = flu.astype(np.float64)
    spec = (np.array([33.3, 61.7, 95.2], np.float32), np.array([2.0, 5.0, 3.0], np.float32))
    eg = GRID.e0_kev + GRID.de_kev * np.arange(GRID.n_e)
    resp = (0.5 * eg + 3.0).astype(np.float32)     # exact in float32
    p = make(ph, g, spec=spec, fluence=flu, response=resp)
    pix = np.arange(g.nu * g.nv)
    S, d, _ = pixel_rays(g, pix)
    half = 0.5 * np.array(ph.shape[::-1]) * np.array(ph.spacing_mm)
    e = spec[0].astype(np.float64)
    mt = np.array([mu_total(ph.materials, ek)[0] for ek in e])
    phi = spec[1].astype(np.float64) / spec[1].astype(np.float64).sum()
    r = 0.5 * e + 3.0
    rho = float(ph.density[0, 0, 0])
    expect = np.zeros(pix.size)
    hits = 0
    for k in pix:
        c = chord(S, d[k], half)
        ln = 0.0 if c is None else c[1] - c[0]
        hits += c is not None
        expect[k] = flu64.ravel()[k] / flu64.sum() * (phi * r * np.exp(-0.1 * rho * mt * ln)).sum()
    assert 0 < hits < pix.size                     # some rays miss the box
    for interp in (True, False):
        for dl in (0.0, 0.37, 5.0):
            got = oracle_lib.primary_raytrace(p, interp=interp, dl=dl).ravel()
            assert np.allclose(got, expect, rtol=1e-10, atol=0), (interp, dl)


@pytest.mark.parametrize("seed,e", [(1, 60.0), (2, 41.3)])
def test_converges_to_the_line_integral_of_the_interpolated_attenuation(oracle_lib, seed, e):
    """Several materials: the sum of dl mu(x_j) with mu interpolated from the
    voxel attenuation coefficients rho_v mu(m_v, E) converges to that field's
    line integral at the rate of the midpoint rule."""
    ph = random_phantom(seed)
    g = W.Geometry(phi_rad=0.3 + seed, theta_rad=0.0, nu=12, nv=10, du_mm=5.0, dv_mm=5.0)
    p = make(ph, g, spec=W.mono_spectrum(e))
    rng = np.random.default_rng(seed + 10)
    S, d, _ = pixel_rays(g, np.arange(g.nu * g.nv))
    half = 0.5 * np.array(ph.shape[::-1]) * np.array(ph.spacing_mm)
    hit = [k for k in range(g.nu * g.nv) if chord(S, d[k], half)]
    pix = rng.choice(hit, 6, replace=False)
    f = mu_field(ph, e, True)
    wk = p.fluence.ravel().astype(np.float64) / p.fluence.astype(np.float64).sum()
    exact = np.array([exact_line_integral(ph, f, S, d[k], chord(S, d[k], half), True) for k in pix])
    for dl, tol in ((0.01, 2e-6), (0.5, 2e-3)):
        got = oracle_lib.primary_raytrace(p, interp=True, dl=dl, pixels=pix)
        L = -10.0 * np.log(got / (wk[pix] * e))
        rel = np.abs(L - exact) / exact
        assert rel.max() < tol, (dl, rel)
    # the default step is half the smallest voxel edge
    a = oracle_lib.primary_raytrace(p, interp=True, dl=0.0, pixels=pix)
    b = oracle_lib.primary_raytrace(p, interp=True, dl=0.5 * min(ph.spacing_mm), pixels=pix)
    assert np.array_equal(a, b)


def test_interpolation_off_is_the_voxel_constant_integral(oracle_lib):
    ph = random_phantom(5)
    e = 70.0
    g = W.Geometry(phi_rad=2.2, nu=12, nv=10, du_mm=5.0, dv_mm=5.0)
    p = make(ph, g, spec=W.mono_spectrum(e))
    S, d, _ = pixel_rays(g, np.arange(g.nu * g.nv))
    half = 0.5 * np.array(ph.shape[::-1]) * np.array(ph.spacing_mm)
    pix = [k for k in range(g.nu * g.nv) if chord(S, d[k], half)][::7][:6]
    f = mu_field(ph, e, False)
    exact = np.array([exact_line_integral(ph, f, S, d[k], chord(S, d[k], half), False) for k in pix])
    got = oracle_lib.primary_raytrace(p, interp=False, dl=2e-4, pixels=pix)
    wk = p.fluence.ravel().astype(np.float64) / p.fluence.astype(np.float64).sum()
    L = -10.0 * np.log(got / (wk[pix] * e))
    assert np.max(np.abs(L - exact) / exact) < 1e-4


def test_agrees_with_the_exact_primary_on_one_material(oracle_lib):
    """With one material, interpolating rho mu and interpolating rho agree, so
    the ray tracer at small dl meets the exact-integral primary evaluated at the
    pixel centres (1-point rule), an independent code path."""
    rng = np.random.default_rng(8)
    shape = (8, 9, 10)
    ph = W.Phantom(rng.uniform(0.5, 1.5, shape).astype(np.float32), np.zeros(shape, np.uint8),
                   (3.0, 2.0, 2.5), ["soft_tissue"])
    g = W.Geometry(phi_rad=1.1, theta_rad=0.05, nu=16, nv=12, du_mm=4.0, dv_mm=4.0)
    spec = (np.array([40.0, 70.0, 100.0], np.float32), np.array([0.3, 0.4, 0.3], np.float32))
    p = make(ph, g, spec=spec)
    a = oracle_lib.primary_raytrace(p, interp=True, dl=0.02)
    b = oracle_lib.primary_exact(p, interp=True, nq=1)
    assert np.allclose(a, b, rtol=2e-6, atol=0)


def test_sphere_is_symmetric(oracle_lib):
    ph = W.sphere_phantom(32, 4.0, 50.0)
    g0 = W.Geometry(phi_rad=0.0, nu=32, nv=24, du_mm=8.0, dv_mm=8.0)
    a = oracle_lib.primary_raytrace(make(ph, g0))
    b = oracle_lib.primary_raytrace(make(ph, g0.replace(phi_rad=0.5 * math.pi)))
    assert np.allclose(a, b, rtol=1e-9)
    assert np.allclose(a, a[:, ::-1], rtol=1e-9)
    assert np.allclose(a, a[::-1, :], rtol=1e-9)


@pytest.mark.parametrize("phi,obj,uv", [
    (0.0, (0.0, 30.0, 20.0), (45.0, 30.0)),
    (0.5 * math.pi, (-30.0, 0.0, -20.0), (45.0, -30.0)),
])
def test_shadow_lands_where_the_geometry_says(oracle_lib, phi, obj, uv):
    n, d = 40, 2.5
    ph = W.box_phantom((n, n, n), (d, d, d), material="air", density=0.0)
    ph = W.Phantom(ph.density, ph.material, ph.spacing_mm, ["air", "bone"])
    c = ((np.arange(n) + 0.5) - n / 2) * d
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    cube = (abs(X - obj[0]) < 5) & (abs(Y - obj[1]) < 5) & (abs(Z - obj[2]) < 5)
    ph.material[cube] = 1
    ph.density[cube] = 1.85
    g = W.Geometry(phi_rad=phi, nu=64, nv=48, du_mm=4.0, dv_mm=4.0)
    p = make(ph, g)
    img = oracle_lib.primary_raytrace(p)
    flu = p.fluence.astype(np.float64) / p.fluence.astype(np.float64).sum() * 60.0
    deficit = 1.0 - img / flu
    uc = (np.arange(g.nu) + 0.5 - g.nu / 2) * g.du_mm
    vc = (np.arange(g.nv) + 0.5 - g.nv / 2) * g.dv_mm
    wsum = deficit.sum()
    cu = (deficit.sum(0) * uc).sum() / wsum
    cv = (deficit.sum(1) * vc).sum() / wsum
    assert abs(cu - uv[0]) < 1.0 and abs(cv - uv[1]) < 1.0


def test_rejects_bad_input(oracle_lib):
    ph = W.box_phantom((4, 4, 4), (2.0, 2.0, 2.0))
    g = W.Geometry(nu=8, nv=6)
    p = make(ph, g)
    with pytest.raises(ValueError):
        oracle_lib.primary_raytrace(p, pixels=[48])
    ph.material[0, 0, 0] = 3                         # beyond the table
    with pytest.raises(ValueError):
        oracle_lib.primary_raytrace(make(ph, g))
