"""The launch-shape autotuner on a small two-phantom batch: the search runs
over every candidate and the refinement stage, writes its cache under a key
that names the kernel sources and the device, is answered from the cache the
second time, and the shape it picks gives the default shape's tallies bit for
bit (tallies are fixed-point sums keyed by photon index); the same for the
adjoint's search."""
import json

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_6367_amd import api
    return api


def small_batch(gpu):
    geom = W.Geometry(nu=48, nv=32, du_mm=8.0, dv_mm=8.0)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    src = W.Source(spec[0], spec[1], W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    phs = [W.ellipsoid_phantom((32, 48, 48), (4.0, 4.0, 4.0), 61, n_inner=6),
           W.ellipsoid_phantom((24, 40, 40), (5.0, 5.0, 5.0), 62, n_inner=6)]
    physw = W.physics_for(phs[0])
    phys = gpu.DevicePhysics(physw.mu_mass, physw.grid.e0_kev, physw.grid.de_kev)
    dsrc = gpu.DeviceSource(src.spec_e, src.spec_p, src.fluence)
    vols = [gpu.DeviceVolume(p.density, p.material, p.spacing_mm).local_majorants(8, 0.1) for p in phs]
    jobs = [gpu.JobSpec(geom.replace(phi_rad=0.5 * k), 400_000, k, volume=k % 2) for k in range(6)]
    jobs.sort(key=lambda j: j.volume)
    return gpu.Batch(vols, phys, [dsrc], jobs)


def test_autotune_search_cache_and_identical_tallies(gpu, tmp_path):
    import torch
    from paper_1204_6367_amd import autotune
    b = small_batch(gpu)
    cache = str(tmp_path / "tune.json")
    best = autotune.autotune(b, fraction=0.5, min_photons=100_000, cache=cache, force=True)
    log("forward best", best)
    table = json.load(open(cache))
    key = autotune.workload_key(b, "forward", True)
    assert key in table and autotune.kernel_sha() in key
    assert table[key]["tuning"] == best
    assert len(table[key]["all"]) >= len(autotune.CANDIDATES)          # every candidate ran, then the refinement
    # answered from the cache
    assert autotune.autotune(b, cache=cache) == best
    ref = b.project(seed=3, sumsq=True)
    got = b.project(seed=3, sumsq=True, tune=best)
    assert torch.equal(got, ref)
    # the adjoint's search, and its shape against the default
    g = b.jobs[0].geom
    adj = torch.tensor(np.random.default_rng(4).normal(size=(len(b.jobs), 2, g.nv, g.nu)), device="cuda")
    bb = autotune.autotune(b, fraction=0.5, min_photons=100_000, cache=cache, force=True, mode="backward",
                           volume=1)
    log("backward best", bb)
    assert autotune.workload_key(b, "backward", True) in json.load(open(cache))
    maj = b.majorants(True, 0.1)
    g0 = b.backward(adj, maj, volume=1, seed=5)
    g1 = b.backward(adj, maj, volume=1, seed=5, tune=bb)
    assert torch.allclose(g1, g0, rtol=1e-9, atol=1e-12 * float(g0.abs().max()))
