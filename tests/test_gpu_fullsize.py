"""Parity at the benchmark's full sizes: for each phantom of the multi-phantom
workload (and the single-projection workload), one job at its full photon
count on the GPU; the oracle recomputes a random sample of its histories one
by one, and the job's tallies from the batched launch must equal the sums of
the traced histories (a property that holds at any size)."""
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


CASES = [
    # (label, phantom builder, photons, phi)
    ("pelvis-256x256x160", lambda: W.ellipsoid_phantom((160, 256, 256), (1.95, 1.95, 2.5), 11), 100_000_000, 0.0),
    ("multi-512x512x256", lambda: W.ellipsoid_phantom(*W.MULTI_PHANTOMS[0][:3]), 100_000_000, 1.3),
    ("multi-256x256x160", lambda: W.ellipsoid_phantom(*W.MULTI_PHANTOMS[1][:3]), 30_000_000, 2.1),
    ("multi-128x128x64", lambda: W.ellipsoid_phantom(*W.MULTI_PHANTOMS[2][:3]), 10_000_000, 4.0),
]


@pytest.mark.parametrize("label,builder,n,phi", CASES, ids=[c[0] for c in CASES])
def test_full_size_job(gpu, label, builder, n, phi):
    import torch
    import oracle
    log("case", label, n)
    ph = builder()
    geom = W.Geometry(**W.PELVIS_DET).replace(phi_rad=phi)
    prob = W.Problem(ph, W.physics_for(ph), W.pelvis_source(geom), geom, n)
    vol, phys, src = gpu.upload(prob)
    jid = 17
    # the batched launch (as the benchmark runs it), with a second volume so the
    # dispenser switches phantoms
    small = W.sphere_phantom(16, 4.0, 20.0)
    small.materials[:] = ["air", "soft_tissue"]
    svol = gpu.DeviceVolume(small.density, small.material, small.spacing_mm)
    jobs = [gpu.JobSpec(geom, n, jid, volume=0), gpu.JobSpec(geom, 1_000_000, jid + 1, volume=1)]
    b = gpu.Batch([vol, svol], phys, [src], jobs)
    tb = b.tally_views(b.project(seed=1))[0].cpu().numpy()
    tr = gpu.trace(vol, phys, src, geom, n, seed=1, job_id=jid)
    rng = np.random.default_rng(99)
    ids = np.sort(rng.choice(n, 3000, replace=False)).astype(np.int64)
    idt = torch.tensor(ids, device="cuda")
    g = {k: v.index_select(0, idt).cpu().numpy() for k, v in tr.items()}
    p = oracle.Problem.from_workload(prob, phi_rad=phi)
    o = oracle.mc_histories(p, 1, ids.astype(np.uint32), oracle.majorant(p), job_id=jid)
    same = (g["cls"].astype(np.int64) == o["cls"]) & (g["pixel"] == o["pixel"]) & \
        (g["n_compton"] == o["n_compton"]) & (g["n_rayleigh"] == o["n_rayleigh"]) & \
        (g["steps"] == o["steps"]) & (np.abs(g["e_final"] - o["e_final"]) <= 2e-4 * o["e_final"])
    log(label, "identical sampled histories", same.mean())
    assert same.mean() >= 0.99
    # tallies of the batched launch = sums of the traced histories
    cls = tr["cls"]
    assert int((cls < 0).sum()) == 0
    npix = geom.nu * geom.nv
    e = tr["e_final"].double()
    q = torch.round(e * 2**20)
    for c, k in ((0, 0), (1, 2)):
        sel = cls == c
        acc = torch.zeros(npix, dtype=torch.float64, device="cuda")
        acc.index_add_(0, tr["pixel"][sel].long(), q[sel])
        acc = (acc / 2**20 / n).view(geom.nv, geom.nu).cpu().numpy()
        assert np.allclose(acc, tb[k], rtol=1e-12, atol=0), (label, c)
