"""Pins of the oracle's path-replay adjoint (score function of delta tracking,
the majorant held fixed) against derivatives of closed-form expectations.
CPU only.

Primary class.  With the adjoint weight 1 on every primary pixel, the loss is
the expected primary energy reaching the detector, and changing the variable
of integration from (aim point, arc length) to position gives
  dL/drho_v = - sum_E phi_E r(E) int dV w_v(x) mu_tot(m(x), E) Phi0(x) T(x, E)
with Phi0 the unattenuated fluence per source photon and T the transmission
of the whole source-to-detector line through x (Eq. 1).  On each cell bounded
by voxel faces and voxel-centre planes w_v is a polynomial and m constant, so a
Gauss rule per cell converges fast.

Scatter class (the real-collision terms).  For a homogeneous box, scaling all
densities by lambda changes the first-order scatter integral; its derivative
at lambda = 1 equals sum_v rho_v dL/drho_v of the first-order scatter tally.
"""
import math

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W
from test_oracle_transport import make, geo_frame, single_scatter_expectation, random_phantom


def primary_gradient_reference(oracle_lib, p, ph, geom, interp, f_area, nq=3):
    nz, ny, nx = ph.density.shape
    sp = np.array(ph.spacing_mm)
    nvox = np.array([nx, ny, nz])
    lo = -0.5 * nvox * sp
    S, P, n, eu, ev = geo_frame(geom.phi_rad, geom.theta_rad, geom.sad_mm, geom.aid_mm)
    t, w = np.polynomial.legendre.leggauss(nq)
    g01, w01 = 0.5 * (t + 1), 0.5 * w
    # sub-cell edges along each axis: faces and centres
    edges = [lo[a] + 0.5 * sp[a] * np.arange(2 * nvox[a] + 1) for a in range(3)]
    mu_tab = p.mu.astype(np.float64)
    egrid = W.EnergyGrid().energies()
    spec_e = p.spec_e.astype(np.float64)
    spec_w = p.spec_p.astype(np.float64) / p.spec_p.astype(np.float64).sum()
    mut = np.array([[np.interp(e, egrid, mu_tab[m].sum(-1)) for m in range(mu_tab.shape[0])]
                    for e in spec_e])                                  # [E][m] cm^2/g
    grad = np.zeros(ph.density.shape)
    pts = []
    for a in range(3):
        e = edges[a]
        pts.append(((e[:-1, None] + (e[1:] - e[:-1])[:, None] * g01[None, :]).ravel(),
                    ((e[1:] - e[:-1])[:, None] * w01[None, :]).ravel()))
    X, Y, Z = np.meshgrid(pts[0][0], pts[1][0], pts[2][0], indexing="ij")
    WX, WY, WZ = np.meshgrid(pts[0][1], pts[1][1], pts[2][1], indexing="ij")
    xs = np.stack([X.ravel(), Y.ravel(), Z.ravel()], -1)
    wv = (WX * WY * WZ).ravel()
    din = xs - S
    r = np.linalg.norm(din, axis=1)
    din /= r[:, None]
    cosn = din @ n
    tD = ((P - S) @ n) / cosn
    D = S + tD[:, None] * din
    phi0 = f_area * tD**2 / cosn / r**2
    ri = oracle_lib.rho_integrals_many(p, S, D + 10.0 * din, interp)   # [Q][m]
    trans = np.exp(-0.1 * ri @ mut.T)                                   # [Q][E]
    gv = (xs - lo) / sp
    iv = np.clip(np.floor(gv).astype(int), 0, nvox - 1)
    m = ph.material[iv[:, 2], iv[:, 1], iv[:, 0]]
    kern = -(spec_w * spec_e * 0.1 * mut[:, m].T * trans).sum(1) * phi0 * wv   # r(E) = E
    if interp:
        gg = gv - 0.5
        k0 = np.floor(gg).astype(int)
        f = gg - k0
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    ww = ((f[:, 0] if bx else 1 - f[:, 0]) * (f[:, 1] if by else 1 - f[:, 1])
                          * (f[:, 2] if bz else 1 - f[:, 2]))
                    ix = np.clip(k0 + np.array([bx, by, bz]), 0, nvox - 1)
                    np.add.at(grad, (ix[:, 2], ix[:, 1], ix[:, 0]), kern * ww)
    else:
        np.add.at(grad, (iv[:, 2], iv[:, 1], iv[:, 0]), kern)
    return grad


@pytest.mark.parametrize("interp", [True, False])
def test_primary_adjoint_matches_volume_integral(oracle_lib, interp):
    shape, sp = (4, 4, 4), (8.0, 8.0, 8.0)
    ph = random_phantom(shape, sp, seed=21)
    g = W.Geometry(nu=8, nv=8, du_mm=20.0, dv_mm=20.0)
    flu = np.zeros((8, 8), np.float32)
    flu[2:6, 2:6] = 1.0                                    # 80 mm field covers the shadow
    p = make(ph, g, fluence=flu)
    # The transmission of the line through x has kinks wherever that line grazes
    # a lattice edge, so the cell rule converges slowly; the reference carries
    # twice the change from 8 to 12 points per axis as its error estimate.
    want = primary_gradient_reference(oracle_lib, p, ph, g, interp, 1.0 / (80.0 * 80.0), nq=12)
    coarse = primary_gradient_reference(oracle_lib, p, ph, g, interp, 1.0 / (80.0 * 80.0), nq=8)
    qerr = 2.0 * np.abs(want - coarse)
    mb = 1.2 * oracle_lib.majorant(p, interp)
    adj = np.zeros((2, 8, 8))
    adj[0] = 1.0
    reps = [oracle_lib.mc_backward(p, s, 400_000, adj, mb, interp=interp) for s in range(1, 9)]
    reps = np.array(reps)
    m = reps.mean(0)
    se = reps.std(0, ddof=1) / math.sqrt(len(reps))
    z = (m - want) / np.sqrt(se**2 + qerr**2)
    assert np.abs(z).max() < 5.0
    assert np.linalg.norm(m - want) / np.linalg.norm(want) < 0.02


def test_primary_adjoint_sign_and_support(oracle_lib):
    """More density anywhere in the beam lowers the primary: every voxel's
    gradient of the total primary is negative; voxels outside the field are 0."""
    shape, sp = (6, 6, 6), (8.0, 8.0, 8.0)
    ph = random_phantom(shape, sp, seed=22)
    g = W.Geometry(nu=8, nv=8, du_mm=20.0, dv_mm=20.0)
    flu = np.zeros((8, 8), np.float32)
    flu[4:6, 4:6] = 1.0                                    # beam through the +u, +v quadrant only
    p = make(ph, g, fluence=flu)
    adj = np.zeros((2, 8, 8))
    adj[0] = 1.0
    gr = oracle_lib.mc_backward(p, 1, 200_000, adj, 1.2 * oracle_lib.majorant(p, False), interp=False)
    assert np.all(gr <= 0) and np.any(gr < 0)
    assert np.all(gr[:, :3, :] == 0) and np.all(gr[:3, :, :] == 0)      # y < 0 or z < 0: unlit


def test_first_order_scatter_adjoint_matches_scaling_derivative(oracle_lib):
    nvox, d = 8, 5.0
    ph = W.box_phantom((nvox, nvox, nvox), (d, d, d), "water", 1.0)
    g = W.Geometry(nu=16, nv=16, du_mm=40.0, dv_mm=40.0)
    flu = np.zeros((16, 16), np.float32)
    flu[7:9, 7:9] = 1.0
    grid = W.EnergyGrid()
    p = make(ph, g, fluence=flu, phys_grid=grid)
    half = np.full(3, 0.5 * nvox * d)
    mu_tab = W.cross_section_table(["water"], grid)[0].astype(np.float64)
    h = 1e-3
    s_plus = single_scatter_expectation(g, half, grid, mu_tab * (1 + h), 1 / 6400.0, 40.0).sum()
    s_minus = single_scatter_expectation(g, half, grid, mu_tab * (1 - h), 1 / 6400.0, 40.0).sum()
    want = (s_plus - s_minus) / (2 * h)
    mb = 1.2 * oracle_lib.majorant(p)
    adj = np.zeros((2, 16, 16))
    adj[1] = 1.0
    reps = np.array([(oracle_lib.mc_backward(p, s, 500_000, adj, mb, mode=1) * ph.density).sum()
                     for s in range(1, 9)])
    m, se = reps.mean(), reps.std(ddof=1) / math.sqrt(len(reps))
    assert abs(m - want) < 4 * se + 3e-3 * abs(want)
    assert se < 0.05 * abs(want)


def test_backward_requires_weights(oracle_lib):
    pr = W.sphere_problem()
    p = oracle_lib.Problem.from_workload(pr)
    mb = oracle_lib.majorant(p)
    g = oracle_lib.mc_backward(p, 1, 10000, np.zeros((2, p.nv, p.nu)), mb)
    assert np.all(g == 0)
