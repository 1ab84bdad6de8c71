"""gdrr_mc_project_static -- the projection without a workspace argument, on
the library's per-device static scratch -- against gdrr_mc_project on the same
arguments: bitwise equal tallies (fixed-point sums), over consecutive calls
whose inputs shrink (the scratch keeps the previous call's contents), with the
library's own majorant and a caller's, and with local majorants."""
import ctypes as C

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


def static_call(gpu, vol, phys, src, geom, n, seed, job_id, flags, out, majorant=None):
    """Straight through the C ABI."""
    import torch
    from paper_1204_6367_amd import _abi
    L = _abi.lib()
    v, p, s, g = vol.struct(), phys.struct(), src.struct(), gpu.geometry_struct(geom)
    mb = None if majorant is None else majorant.data_ptr()
    rc = L.gdrr_mc_project_static(C.byref(v), C.byref(p), C.byref(s), C.byref(g), mb, seed, n, job_id, flags,
                                  out.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    _abi.check(rc)
    return out


def cases():
    big = W.sphere_problem(1_000_000)                                     # 64^3, 64x48 detector
    ph = W.ellipsoid_phantom((40, 48, 56), (3.0, 3.0, 3.0), 5, n_inner=6)
    geom = W.Geometry(phi_rad=1.3, nu=40, nv=30, du_mm=8.0, dv_mm=8.0)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    src = W.Source(spec[0], spec[1], W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    small = W.Problem(ph, W.physics_for(ph), src, geom, 200_003)
    return big, small


@pytest.mark.parametrize("macro", [0, 6])
def test_static_scratch_matches_the_workspace_entry_point(gpu, macro):
    import torch
    from paper_1204_6367_amd import _abi
    flags = _abi.INTERP_DENSITY | _abi.TALLY_SUMSQ
    for k, (prob, seed) in enumerate(zip(cases(), (1, 7))):        # large input first, then a smaller one
        log("static scratch case", k, prob.phantom.shape, prob.n_photons, "macro", macro)
        vol, phys, src = gpu.upload(prob)
        vol.local_majorants(macro)
        g = prob.geom
        want = gpu.project(vol, phys, src, g, prob.n_photons, seed=seed, job_id=3 + k)
        got = torch.full((4, g.nv, g.nu), float("nan"), dtype=torch.float64, device="cuda")
        static_call(gpu, vol, phys, src, g, prob.n_photons, seed, 3 + k, flags, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), k
        # a caller's majorant table (single-majorant tracking only reads it)
        if macro == 0:
            maj = gpu.majorant(vol, phys, True, 0.05)
            want_m = gpu.project(vol, phys, src, g, prob.n_photons, seed=seed, job_id=3 + k, majorant_tab=maj)
            got_m = torch.zeros_like(got)
            static_call(gpu, vol, phys, src, g, prob.n_photons, seed, 3 + k, flags, got_m, majorant=maj)
            torch.cuda.synchronize()
            assert torch.equal(got_m, want_m), k
        assert float(want[0].sum()) > 0.0 and float(want[2].sum()) > 0.0
