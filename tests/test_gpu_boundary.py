"""The boundary on the GPU: invalid device inputs (negative, NaN or infinite
densities; material indices beyond the table; bad source weights) are
transported exactly as their cleaned values (density 0, material n_mat - 1)
and reported by gdrr_input_status; a run split over photon-index ranges and
resumed on the same workspace gives the one-shot run's bits."""
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


def body(seed=3, shape=(24, 32, 40), sp=(4.0, 3.5, 3.0)):
    ph = W.ellipsoid_phantom(shape, sp, seed, n_inner=6)
    geom = W.Geometry(phi_rad=0.4, nu=40, nv=24, du_mm=8.0, dv_mm=8.0)
    spec = W.kramers_spectrum(120.0, 2.5, 2.0)
    src = W.Source(spec[0], spec[1], W.fluence_map(geom, bowtie_mm=30.0, spectrum=spec))
    return W.Problem(ph, W.physics_for(ph), src, geom, 0)


def spoil(ph, n_mat, seed=11):
    """A copy with invalid densities and materials, and its cleaned twin."""
    rng = np.random.default_rng(seed)
    d, m = ph.density.copy(), ph.material.copy()
    flat = d.reshape(-1)
    idx = rng.choice(flat.size, 60, replace=False)
    flat[idx[:20]] = -rng.uniform(0.1, 2.0, 20)
    flat[idx[20:30]] = np.nan
    flat[idx[30:35]] = np.inf
    flat[idx[35:40]] = -np.inf
    mf = m.reshape(-1)
    midx = rng.choice(mf.size, 40, replace=False)
    mf[midx] = rng.integers(n_mat, 256, 40)
    cd = np.where(np.isfinite(d) & (d >= 0), d, 0).astype(np.float32)
    cm = np.minimum(m, n_mat - 1).astype(np.uint8)
    return (d, m), (cd, cm)


@pytest.mark.parametrize("macro", [0, 5])
def test_invalid_inputs_transport_as_cleaned_and_are_reported(gpu, macro):
    import torch
    prob = body()
    ph = prob.phantom
    n_mat = len(ph.materials)
    (bd, bm), (cd, cm) = spoil(ph, n_mat)
    _, phys, src = gpu.upload(prob)
    bad = gpu.DeviceVolume(bd, bm, ph.spacing_mm).local_majorants(macro, 0.1)
    clean = gpu.DeviceVolume(cd, cm, ph.spacing_mm).local_majorants(macro, 0.1)
    jobs = [gpu.JobSpec(prob.geom.replace(phi_rad=a), 200_000, k) for k, a in enumerate((0.4, 2.0))]
    bb = gpu.Batch([bad], phys, [src], jobs)
    bc = gpu.Batch([clean], phys, [src], jobs)
    for interp in (True, False):
        log("forward", macro, interp)
        tb = bb.project(seed=5, interp=interp)
        with pytest.raises(gpu._abi.GdrrError) as e:
            bb.input_status()
        msg = str(e.value)
        assert "densities" in msg and "material" in msg and "weights" not in msg, msg
        tc = bc.project(seed=5, interp=interp)
        bc.input_status()                              # clean inputs: no error
        assert torch.equal(tb, tc)
        # the library's own majorants (computed from the inputs) agree as well
        mb = gpu.majorant(bad, phys, interp, 0.05)
        mc = gpu.majorant(clean, phys, interp, 0.05)
        assert torch.equal(mb, mc)
        # the ray-traced primary (cell records with interpolation, voxels without)
        pb = bb.primary(interp=interp)
        with pytest.raises(gpu._abi.GdrrError):
            gpu.input_status(bb._rt_ws)
        pc = bc.primary(interp=interp)
        gpu.input_status(bc._rt_ws)
        for x, y in zip(pb, pc):
            assert torch.equal(x, y)
    # the adjoint replays the same histories: equal up to the order of float64 atomics
    maj = torch.stack([gpu.majorant(clean, phys, True, 0.2)])
    adj = torch.tensor(np.random.default_rng(2).normal(size=(2, 2, prob.geom.nv, prob.geom.nu)), device="cuda")
    gb = bb.backward(adj, maj, seed=5)
    gc = bc.backward(adj, maj, seed=5)
    assert torch.allclose(gb, gc, rtol=1e-9, atol=1e-12 * float(gc.abs().max()))


def test_bad_source_weights_are_reported(gpu):
    import torch
    prob = body()
    vol, phys, src = gpu.upload(prob)
    zero = gpu.DeviceSource(src.spec_e, torch.zeros_like(src.spec_p), src.fluence)
    b = gpu.Batch([vol], phys, [zero], [gpu.JobSpec(prob.geom, 1000, 0)])
    b.project(seed=1)
    with pytest.raises(gpu._abi.GdrrError) as e:
        b.input_status()
    assert "weights" in str(e.value) and "densities" not in str(e.value)
    neg = gpu.DeviceSource(src.spec_e, src.spec_p, -src.fluence)
    b2 = gpu.Batch([vol], phys, [neg], [gpu.JobSpec(prob.geom, 1000, 0)])
    b2.project(seed=1)
    with pytest.raises(gpu._abi.GdrrError):
        b2.input_status()
    # a clean call on the same workspace clears the report
    b3 = gpu.Batch([vol], phys, [src], [gpu.JobSpec(prob.geom, 1000, 0)])
    b3._ws = b2.workspace()
    b3.project(seed=1)
    b3.input_status()


@pytest.mark.parametrize("macro", [0, 4])
def test_split_and_resumed_run_is_bitwise_the_one_shot_run(gpu, macro):
    """Photon ranges [0, m) then [m, N) with GDRR_RESUME on the same workspace
    equal one call over [0, N), bit for bit (fixed-point sums)."""
    import torch
    prob = body(seed=4)
    vol, phys, src = gpu.upload(prob)
    vol.local_majorants(macro)
    n = 1_000_003
    jobs = [gpu.JobSpec(prob.geom.replace(phi_rad=a), n, 7 + k) for k, a in enumerate((0.1, 1.9, 3.3))]
    one = gpu.Batch([vol], phys, [src], jobs).project(seed=9)
    b = gpu.Batch([vol], phys, [src], jobs)
    cuts = [0, 123_457, 600_001, n]
    for k in range(len(cuts) - 1):
        b.set_photon_ranges(cuts[k], cuts[k + 1] - cuts[k])
        out = b.project(seed=9, resume=k > 0)
        log("resume piece", k, cuts[k], cuts[k + 1])
    assert torch.equal(out, one)
    # uneven cuts per job
    b.set_photon_ranges([0, 0, 0], [500_000, 17, n])
    b.project(seed=9)
    b.set_photon_ranges([500_000, 17, n], [n - 500_000, n - 17, 0])
    assert torch.equal(b.project(seed=9, resume=True), one)
    # without resume, an offset range is its own run (per source photon of that range)
    b.set_photon_ranges(n // 2, n - n // 2)
    half = b.project(seed=9)
    b.set_photon_ranges(0, n // 2)
    first = b.project(seed=9)
    w = torch.tensor([n // 2, n - n // 2], dtype=torch.float64, device="cuda") / n
    assert torch.allclose(w[0] * first + w[1] * half, one, rtol=1e-12, atol=1e-18)


def test_noise_scale_through_the_binding(gpu):
    assert abs(gpu.noise_scale(5e8, 5.2913e9, 1.0) - 0.3074) < 5e-4
    with pytest.raises(gpu._abi.GdrrError):
        gpu.noise_scale(0.0, 1.0, 1.0)
