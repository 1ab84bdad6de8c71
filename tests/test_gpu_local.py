"""GPU parity of tracking with local majorants (cubes of voxels, each with its
own bound) against the CPU oracle's local-majorant transport on the same
Philox streams: histories one by one and tallies, with interpolation on and
off, cubes that do not divide the phantom, a batch mixing a local-majorant
volume with a single-majorant one, the full-size benchmark phantoms on
sampled histories, and the adjoint."""
import sys

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

from test_gpu_parity import compare_histories, tally_parity

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


def body_problem(n, seed=7, shape=(40, 48, 56), spacing=(3.0, 2.5, 2.0), nu=48, nv=32):
    ph = W.ellipsoid_phantom(shape, spacing, seed, n_inner=8)
    geom = W.Geometry(phi_rad=0.6, nu=nu, nv=nv, du_mm=6.0, dv_mm=6.0)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    src = W.Source(spec[0], spec[1], W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    return W.Problem(ph, W.physics_for(ph), src, geom, n)


@pytest.mark.parametrize("macro,interp", [(5, True), (3, False), (16, True)])
def test_local_histories_match_oracle(gpu, macro, interp):
    import oracle
    prob = body_problem(200_000)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(macro)
    log("trace local", macro, interp)
    g = gpu.trace(vol, phys, src, prob.geom, prob.n_photons, seed=4, interp=interp)
    p = oracle.Problem.from_workload(prob).local_majorants(macro)
    o = oracle.mc_project(p, 4, prob.n_photons, interp=interp, trace=True)
    frac, _ = compare_histories(g, o)
    log("identical histories", frac)
    assert frac >= 0.999


def test_local_tallies_match_oracle(gpu):
    import oracle
    prob = body_problem(1_000_000)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(4)
    log("project local n=1e6")
    tg = gpu.project(vol, phys, src, prob.geom, prob.n_photons, seed=2).cpu().numpy()
    p = oracle.Problem.from_workload(prob).local_majorants(4)
    to = oracle.mc_project(p, 2, prob.n_photons)["tally"]
    r = tally_parity(tg, to, prob.n_photons, pool=4)
    log(r)
    for k in ("P", "S"):
        assert r[k]["max_z"] <= 3.0
        assert r[k]["rel_l2"] <= 0.01


def test_mixed_batch_equals_single_projections(gpu):
    """A local-majorant volume and a single-majorant one in one launch give
    bitwise the tallies of their single projections."""
    import torch
    a = body_problem(300_000)
    b = W.sphere_problem(300_000)
    va, pa, sa = gpu.upload(a)
    va.local_majorants(6)
    vb = gpu.DeviceVolume(b.phantom.density, np.where(b.phantom.material > 0, 1, 0).astype(np.uint8),
                          b.phantom.spacing_mm)
    jobs = [gpu.JobSpec(a.geom.replace(phi_rad=p), 300_000, k, volume=k % 2) for k, p in enumerate([0.0, 1.0, 2.0, 3.0])]
    bt = gpu.Batch([va, vb], pa, [sa], jobs)
    out = bt.tally_views(bt.project(seed=3))
    for j, t in zip(jobs, out):
        v = [va, vb][j.volume]
        one = gpu.project(v, pa, sa, j.geom, j.n_photons, seed=3, job_id=j.job_id)
        assert torch.equal(t, one)


def test_untraced_volumes_do_not_change_results(gpu):
    """Cube records are staged only for the volumes a launch traces: a batch
    whose jobs use one of three local-majorant volumes gives bitwise the
    tallies of that volume alone, and the adjoint of one volume of a batch
    equals that of a batch holding it alone (float64 atomics: to 1e-12)."""
    import torch
    a = body_problem(200_000)
    c = body_problem(200_000, seed=9, shape=(30, 40, 44))
    va, pa, sa = gpu.upload(a)
    vc = gpu.DeviceVolume(c.phantom.density, c.phantom.material, c.phantom.spacing_mm)
    vd = gpu.DeviceVolume(c.phantom.density[::-1].copy(), c.phantom.material[::-1].copy(), c.phantom.spacing_mm)
    for v, m in ((va, 5), (vc, 4), (vd, 7)):
        v.local_majorants(m, margin=0.1)
    jobs = [gpu.JobSpec(a.geom.replace(phi_rad=p), 200_000, k, volume=1) for k, p in enumerate([0.3, 1.7])]
    three = gpu.Batch([vc, va, vd], pa, [sa], jobs)
    alone = gpu.Batch([va], pa, [sa], [gpu.JobSpec(j.geom, j.n_photons, j.job_id) for j in jobs])
    log("untraced volumes: forward")
    t3 = three.tally_views(three.project(seed=5))
    t1 = alone.tally_views(alone.project(seed=5))
    for x, y in zip(t3, t1):
        assert torch.equal(x, y)
    log("untraced volumes: adjoint")
    rng = np.random.default_rng(4)
    adj = torch.tensor(rng.normal(size=(len(jobs), 2, a.geom.nv, a.geom.nu)), device="cuda")
    g3 = three.backward(adj, three.majorants(True, 0.1), volume=1, seed=2)
    g1 = alone.backward(adj, alone.majorants(True, 0.1), volume=0, seed=2)
    rel = float((g3 - g1).norm() / g1.norm())
    log("adjoint rel diff", rel)
    assert rel < 1e-12


@pytest.mark.parametrize("idx,macro", [(0, 16), (1, 8), (2, 4)])
def test_full_size_sampled_histories(gpu, idx, macro):
    import torch
    import oracle
    shape, sp, seed, _, nph = W.MULTI_PHANTOMS[idx]
    log("local full size", shape, macro)
    ph = W.ellipsoid_phantom(shape, sp, seed)
    geom = W.Geometry(**W.PELVIS_DET).replace(phi_rad=0.9 + idx)
    prob = W.Problem(ph, W.physics_for(ph), W.pelvis_source(geom), geom, nph)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(macro)
    tr = gpu.trace(vol, phys, src, geom, nph, seed=1, job_id=11)
    rng = np.random.default_rng(5 + idx)
    ids = np.sort(rng.choice(nph, 3000, replace=False)).astype(np.int64)
    idt = torch.tensor(ids, device="cuda")
    g = {k: v.index_select(0, idt) for k, v in tr.items()}
    p = oracle.Problem.from_workload(prob, phi_rad=geom.phi_rad).local_majorants(macro)
    o = oracle.mc_histories(p, 1, ids.astype(np.uint32), None, job_id=11)
    frac, _ = compare_histories(g, o)
    log("identical sampled histories", frac)
    assert frac >= 0.99


def test_local_adjoint_matches_oracle(gpu):
    import torch
    import oracle
    rng = np.random.default_rng(21)
    n3 = (10, 10, 10)
    m = rng.integers(0, 3, n3).astype(np.uint8)
    dens = (np.array([0.0012, 1.03, 1.85])[m] * rng.uniform(0.7, 1.3, n3)).astype(np.float32)
    ph = W.Phantom(dens, m, (5.0, 5.0, 5.0), ["air", "soft_tissue", "bone"])
    geom = W.Geometry(phi_rad=0.3, nu=16, nv=12, du_mm=8.0, dv_mm=8.0)
    spec = (np.array([40.0, 60.0, 80.0], np.float32), np.array([0.3, 0.4, 0.3], np.float32))
    prob = W.Problem(ph, W.physics_for(ph), W.Source(*spec, W.fluence_map(geom)), geom, 200_000)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(3, margin=0.2)
    adj = rng.normal(size=(2, geom.nv, geom.nu))
    b = gpu.Batch([vol], phys, [src], [gpu.JobSpec(geom, prob.n_photons, 0)])
    dummy = torch.zeros(1, phys.n_e - 1, dtype=torch.float32, device="cuda")    # unused with local majorants
    gg = b.backward(torch.tensor(adj[None], device="cuda"), dummy, seed=1).cpu().numpy()
    p = oracle.Problem.from_workload(prob).local_majorants(3, margin=0.2)
    go = oracle.mc_backward(p, 1, prob.n_photons, adj, None)
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    log("local adjoint rel L2", rel)
    assert rel <= 0.02


def test_bad_collision_deferral_rejected(gpu):
    prob = body_problem(1000)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(4)
    b = gpu.Batch([vol], phys, [src], [gpu.JobSpec(prob.geom, 1000, 0)])
    for bad in (-1, 65):
        with pytest.raises(gpu._abi.GdrrError):
            b.project(seed=1, tune=dict(coll_defer=bad))


def test_all_local_launch_shapes_give_the_same_bits(gpu):
    """In the all-local instantiation the LDS holds as many rows of material
    sets as the launch shape leaves room for (none to all; cubes of the other
    sets take their bound from the mask in their global record): tallies are
    bitwise the same for every shape."""
    import torch
    a = body_problem(1)
    ph2 = W.ellipsoid_phantom((30, 36, 40), (4.0, 3.5, 3.0), 9, n_inner=10)
    va, pa, sa = gpu.upload(a)
    vb = gpu.DeviceVolume(ph2.density, ph2.material, ph2.spacing_mm)
    va.local_majorants(5)
    vb.local_majorants(4)
    jobs = [gpu.JobSpec(a.geom.replace(phi_rad=0.4 * k), 60_000 + 531 * k, k, volume=k % 2) for k in range(6)]
    bt = gpu.Batch([va, vb], pa, [sa], jobs)
    ref = bt.project(seed=12)
    for t in (dict(block=64, defer=2, chunk=64), dict(block=256), dict(block=512, coll_defer=20),
              dict(block=1024, blocks_per_cu=1), dict(block=512, blocks_per_cu=3, chunk=128)):
        log("launch shape", t)
        assert torch.equal(bt.project(seed=12, tune=t), ref), t
