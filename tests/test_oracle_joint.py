"""Pins of the oracle's joint source phi(E|u): a spectrum per detector column,
the fuller form of a source defined after a bowtie (Sec. 2.1).  With every row
equal to one spectrum the histories are those of the factorised source; in an
empty phantom the sampled (aim column, energy) pairs follow w(column)
phi_column(E) and the primary equals the closed form w(u) sum_k phi_u,k r(E_k);
the MC primary still matches Eq. 1 exactly integrated; the generator's rows
harden toward the detector edges.  CPU only."""
import math

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

from test_oracle_transport import make, random_phantom, zscores


def column_spectra(nu, seed, n_spec=5):
    rng = np.random.default_rng(seed)
    rows = rng.uniform(0.05, 1.0, (nu, n_spec)).astype(np.float32)
    rows[3, 1:] = 0.0                        # one column carries only the first channel
    return rows


SPEC_E = np.array([30.0, 45.5, 60.0, 80.0, 110.0], np.float32)


def test_identical_rows_give_the_factorised_histories(oracle_lib):
    ph = random_phantom((10, 12, 14), (5.0, 5.0, 5.0), seed=5)
    g = W.Geometry(phi_rad=0.4, nu=12, nv=10, du_mm=10.0, dv_mm=10.0)
    phi = np.array([0.1, 0.3, 0.3, 0.2, 0.1], np.float32)
    a = make(ph, g, spec=(SPEC_E, phi))
    b = make(ph, g, spec=(SPEC_E, np.tile(phi, (g.nu, 1))))
    assert b.s.spec_rows == g.nu
    ids = np.arange(20000)
    mb = oracle_lib.majorant(a)
    ta = oracle_lib.mc_histories(a, 3, ids, mb)
    tb = oracle_lib.mc_histories(b, 3, ids, mb)
    for k in ta:
        assert np.array_equal(ta[k], tb[k]), k
    ra = oracle_lib.mc_project(a, 4, 50000)
    rb = oracle_lib.mc_project(b, 4, 50000)
    assert np.array_equal(ra["tally"], rb["tally"])


def test_empty_phantom_samples_the_joint_pdf(oracle_lib):
    """Zero density: every photon reaches its aim pixel at its source energy, so
    the histogram of (column, channel) is a multinomial draw of
    w(column) phi_column(E) (chi-square over all cells)."""
    ph = W.Phantom(np.zeros((4, 4, 4), np.float32), np.zeros((4, 4, 4), np.uint8), (5.0, 5.0, 5.0), ["water"])
    g = W.Geometry(nu=9, nv=4, du_mm=10.0, dv_mm=10.0)
    rows = column_spectra(g.nu, 2)
    rng = np.random.default_rng(7)
    flu = rng.uniform(0.2, 1.0, (g.nv, g.nu)).astype(np.float32)
    p = make(ph, g, spec=(SPEC_E, rows), fluence=flu)
    n = 400_000
    tr = oracle_lib.mc_histories(p, 9, np.arange(n), oracle_lib.majorant(p))
    assert np.all(tr["cls"] == 0)
    col = tr["pixel"] % g.nu
    ch = np.searchsorted(SPEC_E, tr["e_final"].astype(np.float32))
    assert np.array_equal(SPEC_E[ch], tr["e_final"].astype(np.float32))
    obs = np.zeros((g.nu, len(SPEC_E)))
    np.add.at(obs, (col, ch), 1.0)
    w = flu.astype(np.float64).sum(0) / flu.astype(np.float64).sum()
    r = rows.astype(np.float64) / rows.sum(1, keepdims=True)
    exp = n * w[:, None] * r
    assert np.all(obs[exp == 0.0] == 0.0)          # never a channel the column lacks
    live = exp > 0.0
    chi2 = (((obs - exp) ** 2)[live] / exp[live]).sum()
    dof = live.sum() - 1
    assert abs(chi2 - dof) < 5.0 * math.sqrt(2.0 * dof), (chi2, dof)


@pytest.mark.parametrize("fn", ["exact", "raytrace"])
def test_empty_phantom_primary_closed_form(oracle_lib, fn):
    """P(u) = w(u) sum_k phi_{col(u),k} r(E_k) with nothing in the way: the
    row is chosen by the column (nu != nv, distinct rows)."""
    ph = W.Phantom(np.zeros((4, 4, 4), np.float32), np.zeros((4, 4, 4), np.uint8), (5.0, 5.0, 5.0), ["water"])
    g = W.Geometry(phi_rad=1.1, nu=9, nv=5, du_mm=10.0, dv_mm=10.0)
    rows = column_spectra(g.nu, 4)
    flu = np.random.default_rng(3).uniform(0.2, 1.0, (g.nv, g.nu)).astype(np.float32)
    resp = np.linspace(0.5, 1.5, len(W.EnergyGrid().energies())).astype(np.float32)
    p = make(ph, g, spec=(SPEC_E, rows), fluence=flu, response=resp)
    got = oracle_lib.primary_exact(p, nq=2) if fn == "exact" else oracle_lib.primary_raytrace(p)
    eg = W.EnergyGrid().energies()
    r_e = np.interp(SPEC_E.astype(np.float64), eg, resp.astype(np.float64))
    per_col = (rows.astype(np.float64) * r_e).sum(1) / rows.astype(np.float64).sum(1)
    want = flu.astype(np.float64) / flu.astype(np.float64).sum() * per_col[None, :]
    assert np.allclose(got, want, rtol=1e-12, atol=0.0)


def test_joint_mc_primary_matches_exact_eq1(oracle_lib):
    ph = random_phantom((12, 12, 12), (5.0, 5.0, 5.0), seed=13)
    g = W.Geometry(phi_rad=0.3, nu=16, nv=12, du_mm=8.0, dv_mm=8.0)
    rows = column_spectra(g.nu, 6)
    p = make(ph, g, spec=(SPEC_E, rows))
    want = oracle_lib.primary_exact(p, interp=True, nq=32)
    n = 2_000_000
    r = oracle_lib.mc_project(p, seed=5, n=n)
    z = zscores(r["tally"][0], r["tally"][1], n, want)
    assert np.abs(z).max() < 4.5
    assert abs((z**2).mean() - 1.0) < 0.35
    # the same phantom with the column-averaged spectrum differs far beyond noise
    w = p.fluence.astype(np.float64).sum(0)
    avg = (w[:, None] * rows / rows.sum(1, keepdims=True)).sum(0).astype(np.float32)
    other = oracle_lib.primary_exact(make(ph, g, spec=(SPEC_E, avg)), interp=True, nq=32)
    assert np.abs(zscores(r["tally"][0], r["tally"][1], n, other)).max() > 10.0


def test_joint_table_shape_is_checked(oracle_lib):
    ph = W.box_phantom((4, 4, 4), (5.0, 5.0, 5.0))
    g = W.Geometry(nu=8, nv=6)
    with pytest.raises(ValueError):
        make(ph, g, spec=(SPEC_E, np.ones((g.nv, 5), np.float32)))
    p = make(ph, g, spec=(SPEC_E, np.ones((g.nu, 5), np.float32)))
    p.s.spec_rows = g.nu - 1                    # the C side refuses a table that is not [nu][n_spec]
    with pytest.raises(ValueError):
        oracle_lib.mc_project(p, 1, 10)
    rows = np.ones((g.nu, 5), np.float32)
    rows[2] = 0.0                               # a column with no spectrum
    with pytest.raises(ValueError):
        oracle_lib.mc_project(make(ph, g, spec=(SPEC_E, rows)), 1, 10)


def test_bowtie_rows_harden_toward_the_edges():
    """The generator's rows: each sums to 1, the mean energy rises from the
    centre column to the edges (more aluminium), symmetric about the centre,
    and the fluence-weighted mix of the rows reweights phi(E) by the
    column-averaged transmission, which favours high energies."""
    g = W.Geometry(**W.PELVIS_DET)
    spec = W.kramers_spectrum(120.0, 2.5, 1.0)
    rows = W.bowtie_spectra(g, 30.0, spec).astype(np.float64)
    assert rows.shape == (g.nu, len(spec[0]))
    assert np.allclose(rows.sum(1), 1.0, atol=1e-6)
    mean_e = rows @ spec[0].astype(np.float64)
    c = g.nu // 2
    assert np.all(np.diff(mean_e[c:]) > 0.0) and np.all(np.diff(mean_e[:c]) < 0.0)
    assert np.allclose(mean_e, mean_e[::-1], rtol=1e-5)          # column iu mirrors column nu-1-iu
    phi = spec[1].astype(np.float64) / spec[1].sum()
    assert abs(mean_e[c] - phi @ spec[0]) < 0.5           # the centre column sees almost no aluminium
    assert mean_e[0] > mean_e[c] + 15.0
    flu = W.fluence_map(g, 30.0, spec).astype(np.float64).sum(0)
    mix = (flu[:, None] * rows).sum(0)
    assert mix @ spec[0] > phi @ spec[0] + 2.0
    # bowtie_mm = 0 keeps phi(E) in every column
    flat = W.bowtie_spectra(g, 0.0, spec).astype(np.float64)
    assert np.allclose(flat, phi[None, :], rtol=1e-6)
