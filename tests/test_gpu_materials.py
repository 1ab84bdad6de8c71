"""GPU parity with the largest material count (16, the cell records' 4-bit
material code fully used): histories of the transport (single and local
majorants) and the ray-traced primary against the CPU oracle, on a phantom of
3-voxel blocks of random materials, so that cells of one material -- every id
up to 15 -- and cells mixing materials both occur."""
import sys

import numpy as np
import pytest

from paper_1204_6367_amd import workloads as W

from test_gpu_parity import compare_histories
from test_gpu_raytrace import check_image

pytestmark = pytest.mark.gpu

NAMES = ["air", "water", "soft_tissue", "lung", "bone", "aluminium"]


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


def sixteen_material_problem(n, seed=5, shape=(21, 24, 27), spacing=(3.0, 2.5, 2.0)):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    blocks = rng.integers(0, 16, ((nz + 2) // 3, (ny + 2) // 3, (nx + 2) // 3)).astype(np.uint8)
    mat = np.repeat(np.repeat(np.repeat(blocks, 3, 0), 3, 1), 3, 2)[:nz, :ny, :nx].copy()
    names = [NAMES[k % len(NAMES)] for k in range(16)]
    base = np.array([W.MATERIALS[nm].density for nm in names])
    dens = (base[mat] * rng.uniform(0.7, 1.3, shape)).astype(np.float32)
    ph = W.Phantom(dens, mat, spacing, names)
    grid = W.EnergyGrid()
    # materials that repeat a name get scaled tables, so that all 16 differ
    mu = W.cross_section_table(names, grid) * (1.0 + 0.04 * np.arange(16, dtype=np.float32))[:, None, None]
    phys = W.Physics(mu.astype(np.float32), grid, None)
    geom = W.Geometry(phi_rad=0.4, nu=40, nv=30, du_mm=6.0, dv_mm=6.0)
    spec = W.kramers_spectrum(120.0, 2.5, 4.0)
    src = W.Source(spec[0], spec[1], W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    return W.Problem(ph, phys, src, geom, n)


@pytest.mark.parametrize("macro", [0, 4])
def test_sixteen_materials_histories(gpu, macro):
    import oracle
    prob = sixteen_material_problem(200_000)
    assert set(np.unique(prob.phantom.material)) == set(range(16))
    vol, phys, src = gpu.upload(prob)
    p = oracle.Problem.from_workload(prob)
    if macro:
        vol.local_majorants(macro)
        p.local_majorants(macro)
    log("sixteen materials, macro", macro)
    g = gpu.trace(vol, phys, src, prob.geom, prob.n_photons, seed=6)
    o = oracle.mc_project(p, 6, prob.n_photons, trace=True)
    frac, _ = compare_histories(g, o)
    log("identical histories", frac)
    assert frac >= 0.999


@pytest.mark.parametrize("interp", [True, False])
def test_sixteen_materials_raytrace(gpu, interp):
    import oracle
    prob = sixteen_material_problem(0)
    vol, phys, src = gpu.upload(prob)
    log("sixteen materials ray tracer", interp)
    g = gpu.primary(vol, phys, src, prob.geom, interp=interp).cpu().numpy()
    o = oracle.primary_raytrace(oracle.Problem.from_workload(prob), interp=interp)
    check_image(g, o, f"sixteen materials interp={interp}")
