"""GPU parity of the joint source phi(E|u) -- one spectrum per detector column,
as behind a bowtie that hardens the beam toward the fan's edges -- against the
CPU oracle on the same Philox streams: histories one by one (single and local
majorants, interpolation on and off), tallies, equal rows reproducing the
factorised source bit for bit, a batch mixing a joint and a factorised source,
the ray-traced primary with per-column channel weights, the adjoint, and the
full-size pelvis workload on sampled histories and pixels."""
import sys

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

from test_gpu_parity import compare_histories, tally_parity
from test_gpu_raytrace import check_image

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_6367_amd import api
    return api


def joint_problem(n, seed=7, shape=(40, 48, 56), spacing=(3.0, 2.5, 2.0), nu=48, nv=32, random_rows=False):
    ph = W.ellipsoid_phantom(shape, spacing, seed, n_inner=8)
    geom = W.Geometry(phi_rad=0.6, nu=nu, nv=nv, du_mm=6.0, dv_mm=6.0)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    rows = W.bowtie_spectra(geom, 30.0, spec)
    if random_rows:                                   # rows far apart, some channels absent in some columns
        rng = np.random.default_rng(seed)
        rows = (rows * rng.uniform(0.0, 2.0, rows.shape) * (rng.random(rows.shape) > 0.2)).astype(np.float32)
        rows[:, len(spec[0]) // 2] += 0.01
    src = W.Source(spec[0], rows, W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    return W.Problem(ph, W.physics_for(ph), src, geom, n)


@pytest.mark.parametrize("macro,interp,random_rows", [(0, True, False), (0, False, True), (5, True, True)])
def test_joint_histories_match_oracle(gpu, macro, interp, random_rows):
    import oracle
    prob = joint_problem(200_000, random_rows=random_rows)
    vol, phys, src = gpu.upload(prob)
    p = oracle.Problem.from_workload(prob)
    assert p.s.spec_rows == prob.geom.nu
    if macro:
        vol.local_majorants(macro)
        p.local_majorants(macro)
    log("trace joint source", macro, interp, random_rows)
    g = gpu.trace(vol, phys, src, prob.geom, prob.n_photons, seed=4, interp=interp)
    o = oracle.mc_project(p, 4, prob.n_photons, interp=interp, trace=True)
    frac, _ = compare_histories(g, o)
    log("identical histories", frac)
    assert frac >= 0.999


def test_joint_tallies_match_oracle(gpu):
    import oracle
    prob = joint_problem(1_000_000, random_rows=True)
    vol, phys, src = gpu.upload(prob)
    log("project joint n=1e6")
    tg = gpu.project(vol, phys, src, prob.geom, prob.n_photons, seed=2).cpu().numpy()
    to = oracle.mc_project(oracle.Problem.from_workload(prob), 2, prob.n_photons)["tally"]
    r = tally_parity(tg, to, prob.n_photons, pool=4)
    log(r)
    for k in ("P", "S"):
        assert r[k]["max_z"] <= 3.0
        assert r[k]["rel_l2"] <= 0.01


def test_equal_rows_reproduce_the_factorised_source(gpu):
    """Every row = phi(E): the same histories and bitwise the same tallies and
    ray-traced primary as the one-spectrum source."""
    import torch
    prob = joint_problem(300_000)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    vol, phys, _ = gpu.upload(prob)
    flu = prob.source.fluence
    one = gpu.DeviceSource(spec[0], spec[1], flu)
    rows = gpu.DeviceSource(spec[0], np.tile(spec[1], (prob.geom.nu, 1)), flu)
    log("equal rows")
    a = gpu.project(vol, phys, one, prob.geom, prob.n_photons, seed=6)
    b = gpu.project(vol, phys, rows, prob.geom, prob.n_photons, seed=6)
    assert torch.equal(a, b)
    ta = gpu.trace(vol, phys, one, prob.geom, 50_000, seed=6)
    tb = gpu.trace(vol, phys, rows, prob.geom, 50_000, seed=6)
    for k in ta:
        assert torch.equal(ta[k], tb[k]), k
    ra = gpu.primary(vol, phys, one, prob.geom)
    rb = gpu.primary(vol, phys, rows, prob.geom)
    assert torch.equal(ra, rb)


def test_batch_mixing_joint_and_factorised_sources(gpu):
    """Jobs alternating between a joint and a one-spectrum source in one launch
    give bitwise the tallies of their single projections."""
    import torch
    prob = joint_problem(200_000, random_rows=True)
    vol, phys, sj = gpu.upload(prob)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    sf = gpu.DeviceSource(spec[0], spec[1], prob.source.fluence)
    srcs = [sj, sf]
    jobs = [gpu.JobSpec(prob.geom.replace(phi_rad=p), 200_000, k, source=k % 2) for k, p in enumerate([0.0, 1.0, 2.0, 3.0])]
    bt = gpu.Batch([vol], phys, srcs, jobs)
    out = bt.tally_views(bt.project(seed=3))
    for j, t in zip(jobs, out):
        one = gpu.project(vol, phys, srcs[j.source], j.geom, j.n_photons, seed=3, job_id=j.job_id)
        assert torch.equal(t, one)


@pytest.mark.parametrize("interp", [True, False])
def test_joint_raytrace_matches_oracle(gpu, interp):
    import oracle
    prob = joint_problem(0, random_rows=True)
    grid = W.EnergyGrid()
    resp = (0.9 * (grid.e0_kev + grid.de_kev * np.arange(grid.n_e)) ** 0.95).astype(np.float32)
    prob.physics = W.physics_for(prob.phantom, grid, resp)
    vol, phys, src = gpu.upload(prob)
    log("raytrace joint", interp)
    g = gpu.primary(vol, phys, src, prob.geom, interp=interp).cpu().numpy()
    o = oracle.primary_raytrace(oracle.Problem.from_workload(prob), interp=interp)
    check_image(g, o, f"joint interp={interp}")


def test_joint_adjoint_matches_oracle(gpu):
    import torch
    import oracle
    rng = np.random.default_rng(23)
    n3 = (10, 10, 10)
    m = rng.integers(0, 3, n3).astype(np.uint8)
    dens = (np.array([0.0012, 1.03, 1.85])[m] * rng.uniform(0.7, 1.3, n3)).astype(np.float32)
    ph = W.Phantom(dens, m, (5.0, 5.0, 5.0), ["air", "soft_tissue", "bone"])
    geom = W.Geometry(phi_rad=0.3, nu=16, nv=12, du_mm=8.0, dv_mm=8.0)
    e = np.array([40.0, 60.0, 80.0], np.float32)
    rows = rng.uniform(0.05, 1.0, (geom.nu, 3)).astype(np.float32)
    prob = W.Problem(ph, W.physics_for(ph), W.Source(e, rows, W.fluence_map(geom)), geom, 200_000)
    vol, phys, src = gpu.upload(prob)
    adj = rng.normal(size=(2, geom.nv, geom.nu))
    b = gpu.Batch([vol], phys, [src], [gpu.JobSpec(geom, prob.n_photons, 0)])
    p = oracle.Problem.from_workload(prob)
    log("joint adjoint")
    maj = gpu.majorant(vol, phys, True, margin=0.2)[None]
    gg = b.backward(torch.tensor(adj[None], device="cuda"), maj, seed=1).cpu().numpy()
    go = oracle.mc_backward(p, 1, prob.n_photons, adj, oracle.majorant(p, True, margin=0.2))
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    log("joint adjoint rel L2", rel)
    assert rel <= 0.02


@pytest.mark.parametrize("interp", [True, False])
def test_joint_local_first_order_tallies(gpu, interp):
    """The variants together: a joint source, local majorants, the first-order
    and first-order-Compton scatter tallies, interpolation on and off, against
    the oracle's tallies (pooled rel L2, totals)."""
    import oracle
    prob = joint_problem(600_000, random_rows=True)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(6)
    p = oracle.Problem.from_workload(prob).local_majorants(6)
    n = prob.n_photons
    for flag, mode in ((gpu.SCATTER_FIRST, 1), (gpu.SCATTER_FIRST_COMPTON, 2)):
        log("joint local first order", flag, interp)
        tg = gpu.project(vol, phys, src, prob.geom, n, seed=12, flags=flag, interp=interp).cpu().numpy()
        to = oracle.mc_project(p, 12, n, mode=mode, interp=interp)["tally"]
        r = tally_parity(tg, to, n, pool=8)
        log(r)
        assert r["P"]["rel_l2"] <= 0.01 and r["S"]["rel_l2"] <= 0.03
        assert abs(tg[2].sum() - to[2].sum()) <= 0.01 * to[2].sum()


def test_full_size_pelvis_joint_source(gpu):
    """The pelvis workload (256 x 256 x 160, 256 x 192 detector, 1e8 photons)
    with the bowtie-hardened joint source: 3000 sampled histories against the
    oracle, and 300 sampled ray-traced pixels."""
    import torch
    import oracle
    prob = W.pelvis_problem()
    prob.source = W.pelvis_source(prob.geom, joint=True)
    vol, phys, src = gpu.upload(prob)
    p = oracle.Problem.from_workload(prob)
    log("full-size pelvis joint: trace 1e8")
    tr = gpu.trace(vol, phys, src, prob.geom, prob.n_photons, seed=1, job_id=5)
    rng = np.random.default_rng(17)
    ids = np.sort(rng.choice(prob.n_photons, 3000, replace=False)).astype(np.int64)
    idt = torch.tensor(ids, device="cuda")
    g = {k: v.index_select(0, idt) for k, v in tr.items()}
    del tr
    o = oracle.mc_histories(p, 1, ids.astype(np.uint32), oracle.majorant(p), job_id=5)
    frac, _ = compare_histories(g, o)
    log("identical sampled histories", frac)
    assert frac >= 0.99
    log("full-size pelvis joint: ray tracer")
    img = gpu.primary(vol, phys, src, prob.geom).cpu().numpy().ravel()
    pix = np.sort(rng.choice(img.size, 300, replace=False)).astype(np.int32)
    want = oracle.primary_raytrace(p, pixels=pix)
    err = np.abs(img[pix] - want) / want
    log("ray tracer sampled max rel err", float(err.max()))
    assert err.max() < 1e-4
