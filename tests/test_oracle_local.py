"""Pins of the oracle's local majorants (Woodcock tracking with a bound that
varies from cube to cube): the MC primary still equals Eq. 1 exactly
integrated, for interpolation on and off and cubes that do not divide the
phantom; the bound holds at random positions, including next to cube faces and
where light high-Z voxels touch dense low-Z ones; tallies agree with the global
majorant's; the primary adjoint still matches the volume integral; and the
local bound does cut the number of flights.  CPU only."""
import math

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

from test_oracle_adjoint import primary_gradient_reference
from test_oracle_transport import make, random_phantom, zscores


def bone_water(seed, shape=(10, 10, 10), sp=(5.0, 5.0, 5.0)):
    rng = np.random.default_rng(seed)
    m = (rng.random(shape) < 0.5).astype(np.uint8)
    d = np.where(m == 0, 1.5, 0.2).astype(np.float32)
    return W.Phantom(d, m, sp, ["water", "bone"])


@pytest.mark.parametrize("interp,macro,rho_min", [(True, 1, 0.0), (True, 5, 0.0), (False, 3, 0.0), (True, 4, 0.6)])
def test_local_primary_matches_exact_eq1(oracle_lib, interp, macro, rho_min):
    ph = random_phantom((12, 12, 12), (5.0, 5.0, 5.0), seed=11)
    g = W.Geometry(phi_rad=0.7, nu=16, nv=12, du_mm=8.0, dv_mm=8.0)
    spec = (np.array([30.0, 45.5, 60.0, 80.0, 110.0], np.float32),
            np.array([0.1, 0.3, 0.3, 0.2, 0.1], np.float32))
    p = make(ph, g, spec=spec)
    want = oracle_lib.primary_exact(p, interp=interp, nq=32)
    p.local_majorants(macro, rho_min=rho_min)
    n = 2_000_000
    r = oracle_lib.mc_project(p, seed=3, n=n, interp=interp)
    z = zscores(r["tally"][0], r["tally"][1], n, want)
    assert np.abs(z).max() < 4.5
    assert abs((z**2).mean() - 1.0) < 0.35


def test_local_primary_unbiased_when_light_bone_touches_dense_water(oracle_lib):
    ph = bone_water(32)
    g = W.Geometry(phi_rad=0.2, nu=16, nv=12, du_mm=8.0, dv_mm=8.0)
    p = make(ph, g)
    want = oracle_lib.primary_exact(p, interp=True, nq=32)
    p.local_majorants(3)
    n = 1_000_000
    r = oracle_lib.mc_project(p, seed=8, n=n)
    z = zscores(r["tally"][0], r["tally"][1], n, want)
    assert np.abs(z).max() < 4.5
    assert abs((z**2).mean() - 1.0) < 0.35


def test_local_bound_holds_everywhere(oracle_lib):
    """mu(x, E) <= mbar_B(E) of the cube holding x, at random positions and at
    positions within 1e-9 mm of cube faces, with interpolation on and off."""
    rng = np.random.default_rng(41)
    grid = W.EnergyGrid()
    eg = grid.energies()
    # light cubes whose first outside voxel is dense: positions within half a voxel of
    # the shared face interpolate that voxel, so the bound needs the ring around each cube
    slab = np.full((8, 8, 8), 0.1, np.float32)
    slab[:, :, 4] = 3.0
    slab[4, :, :] = 3.0
    slab_ph = W.Phantom(slab, np.zeros((8, 8, 8), np.uint8), (4.0, 4.0, 4.0), ["water"])
    for ph, macro in ((random_phantom((9, 10, 11), (4.0, 5.0, 3.0), seed=12), 3), (bone_water(33), 4),
                      (slab_ph, 4)):
        p = make(ph, W.Geometry(nu=8, nv=6)).local_majorants(macro)
        tab = p.mu.astype(np.float64).sum(-1)
        nz, ny, nx = ph.density.shape
        sp = np.array(ph.spacing_mm)
        ext = 0.5 * np.array([nx, ny, nz]) * sp
        x = rng.uniform(-ext, ext, (30000, 3))
        # move a third of the points onto cube faces, nudged by +-1e-9 mm
        face = macro * sp
        k = np.arange(len(x)) % 3 == 0
        ax = rng.integers(0, 3, len(x))
        for a in range(3):
            sel = k & (ax == a)
            q = np.round((x[sel, a] + ext[a]) / face[a]) * face[a] - ext[a]
            x[sel, a] = np.clip(q + rng.choice([-1e-9, 1e-9], sel.sum()), -ext[a], ext[a])
        e = rng.uniform(eg[0], eg[-1], len(x))
        mb = oracle_lib.local_majorant_at(p, x, e)
        iv = np.clip(np.floor((x + ext) / sp).astype(int), 0, [nx - 1, ny - 1, nz - 1])
        m = ph.material[iv[:, 2], iv[:, 1], iv[:, 0]]
        mut = np.array([np.interp(e[q], eg, tab[m[q]]) for q in range(len(x))])
        for interp in (True, False):
            rho = oracle_lib.density_at(p, x, interp)
            assert np.all(rho * mut <= mb), interp


def test_local_bound_density_floor(oracle_lib):
    """With a density floor a cube's bound is (1 + margin) max(rho_max, floor)
    max_m mu_tot(m, E), the density factor rounded up to 19 significant bits:
    a cube of air alone takes the floor, a denser cube keeps its own bound, and
    the floor never lowers a bound."""
    ulp19 = 2.0**-18

    def close_above(got, want):
        return np.all(got >= want * (1 - 1e-15)) and np.all(got <= want * (1 + ulp19) * (1 + 1e-15))

    d = np.full((8, 8, 8), 0.0012, np.float32)
    d[4:, :, :] = 1.0
    m = np.zeros((8, 8, 8), np.uint8)
    m[4:, :, :] = 1
    ph = W.Phantom(d, m, (4.0, 4.0, 4.0), ["air", "water"])
    p = make(ph, W.Geometry(nu=8, nv=6))
    tab = p.mu.astype(np.float64).sum(-1)
    eg = W.EnergyGrid().energies()
    e = np.array([20.0, 60.25, 100.0])
    air_pt = np.array([[-10.0, -10.0, -14.0]] * 3)        # cube z in [-16, -8): voxels z 0..1 (+1 ring) are air
    water_pt = np.array([[-10.0, -10.0, 12.0]] * 3)
    for margin in (2.0**-20, 0.1):
        p.local_majorants(2, margin=margin)
        a0 = oracle_lib.local_majorant_at(p, air_pt, e)
        w0 = oracle_lib.local_majorant_at(p, water_pt, e)
        p.local_majorants(2, margin=margin, rho_min=0.05)
        a1 = oracle_lib.local_majorant_at(p, air_pt, e)
        w1 = oracle_lib.local_majorant_at(p, water_pt, e)
        air_tot = np.array([np.interp(x, eg, tab[0]) for x in e])
        water_tot = np.array([np.interp(x, eg, tab[1]) for x in e])
        assert close_above(a0, (1 + margin) * np.float64(np.float32(0.0012)) * air_tot)
        assert close_above(a1, (1 + margin) * 0.05 * air_tot)
        assert np.array_equal(w1, w0) and close_above(w0, (1 + margin) * 1.0 * water_tot)
    p.local_majorants(2, rho_min=-0.01)
    with pytest.raises(ValueError):
        oracle_lib.mc_project(p, 1, 10)


def test_local_bound_is_the_chord_of_the_node_maxima(oracle_lib):
    """Within an energy interval a mixed cube's bound follows the chord between
    the largest mu_tot of its materials at the interval's two grid energies,
    which lies above the larger of the materials' own lines where those cross
    inside the interval.  A hand-made table of two materials (mu_tot 4, 2, 1,
    1, 1 and 1, 3, 1, 2, 0.5 cm^2/g at 20 ... 60 keV), density 1 everywhere and
    margin 2^-20, whose density factor 1 + 2^-20 rounds up to 1 + 2^-18 at 19
    significant bits: bound / (1 + 2^-18) = 4, 3.5, 3, 2, 1, 1.5, 2, 1.5, 1
    at 20, 25, ..., 60 keV (the larger line alone would give 3.0 at 25 keV and
    1.25 at 55 keV)."""
    import oracle
    mu = np.zeros((2, 5, 3), np.float32)
    mu[0, :, 1] = [4.0, 2.0, 1.0, 1.0, 1.0]
    mu[1, :, 1] = [1.0, 3.0, 1.0, 2.0, 0.5]
    mat = np.zeros((4, 4, 4), np.uint8)
    mat[:, :, 2:] = 1
    g = W.Geometry(nu=8, nv=6)
    p = oracle.Problem(np.ones((4, 4, 4), np.float32), mat, (5.0, 5.0, 5.0), mu, 20.0, 10.0,
                       np.array([40.0], np.float32), np.array([1.0], np.float32), W.fluence_map(g),
                       g.sad_mm, g.aid_mm, g.phi_rad, g.theta_rad, g.nu, g.nv, g.du_mm, g.dv_mm, e_cut_kev=20.0)
    p.local_majorants(4)                                   # one cube holding both materials
    e = 20.0 + 5.0 * np.arange(9)
    got = oracle_lib.local_majorant_at(p, np.zeros((len(e), 3)), e) / (1.0 + 2.0**-18)
    assert np.array_equal(got, [4.0, 3.5, 3.0, 2.0, 1.0, 1.5, 2.0, 1.5, 1.0])


def test_local_and_global_tallies_agree(oracle_lib):
    """Primary and scatter tallies of the two majorants agree within noise on a
    heterogeneous phantom (pooled 4 x 4 bins and totals)."""
    ph = W.ellipsoid_phantom((24, 32, 32), (4.0, 4.0, 4.0), seed=7, n_inner=6)
    g = W.Geometry(phi_rad=0.3, nu=32, nv=24, du_mm=8.0, dv_mm=8.0)
    spec = W.kramers_spectrum(120.0, 2.5, 4.0)
    p = make(ph, g, spec=spec)
    n = 2_000_000
    a = oracle_lib.mc_project(p, 1, n)
    p.local_majorants(4)
    b = oracle_lib.mc_project(p, 2, n)
    assert b["stats"]["steps"] < 0.5 * a["stats"]["steps"]
    for k in (0, 2):
        ta, tb = a["tally"][k], b["tally"][k]
        va = np.maximum(a["tally"][k + 1] - ta**2, 0) / n
        vb = np.maximum(b["tally"][k + 1] - tb**2, 0) / n
        pool = lambda x: x.reshape(6, 4, 8, 4).sum(axis=(1, 3))
        z = (pool(ta) - pool(tb)) / np.sqrt(pool(va) + pool(vb) + 1e-300)
        assert np.abs(z).max() < 4.5, k
        tot = (ta.sum() - tb.sum()) / math.sqrt(va.sum() + vb.sum())
        assert abs(tot) < 4.0, k


def test_local_adjoint_matches_volume_integral(oracle_lib):
    shape, sp = (4, 4, 4), (8.0, 8.0, 8.0)
    ph = random_phantom(shape, sp, seed=21)
    g = W.Geometry(nu=8, nv=8, du_mm=20.0, dv_mm=20.0)
    flu = np.zeros((8, 8), np.float32)
    flu[2:6, 2:6] = 1.0
    p = make(ph, g, fluence=flu)
    want = primary_gradient_reference(oracle_lib, p, ph, g, True, 1.0 / (80.0 * 80.0), nq=12)
    coarse = primary_gradient_reference(oracle_lib, p, ph, g, True, 1.0 / (80.0 * 80.0), nq=8)
    qerr = 2.0 * np.abs(want - coarse)
    p.local_majorants(2, margin=0.2, rho_min=0.3)
    adj = np.zeros((2, 8, 8))
    adj[0] = 1.0
    reps = np.array([oracle_lib.mc_backward(p, s, 400_000, adj, None) for s in range(1, 9)])
    m = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(len(reps))
    z = (m - want) / np.sqrt(se**2 + qerr**2)
    assert np.abs(z).max() < 5.0
    assert np.linalg.norm(m - want) / np.linalg.norm(want) < 0.03


def test_local_majorant_needs_no_table_and_rejects_bad_cubes(oracle_lib):
    ph = W.box_phantom((6, 6, 6), (4.0, 4.0, 4.0))
    p = make(ph, W.Geometry(nu=8, nv=6)).local_majorants(2)
    r = oracle_lib.mc_project(p, 1, 1000)                  # no global table needed
    assert sum(r["stats"]["classes"].values()) == 1000
    p.local_majorants(-1)
    with pytest.raises(ValueError):
        oracle_lib.mc_project(p, 1, 10)
