"""The C ABI without a GPU: the library loads, exports every function the
header declares, its structs have the layout the binding assumes, and
invalid arguments are rejected on the host with a message."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gdrr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gdrr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_1204_6367_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build()
    return _abi


def test_library_exports_every_declared_function(abi):
    names = declared_functions()
    assert len(names) >= 10
    L = abi.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(abi.SIGNATURES)


LAYOUT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "gdrr.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
    printf("gdrr_volume %zu\n", sizeof(gdrr_volume));
    printf("gdrr_physics %zu\n", sizeof(gdrr_physics));
    printf("gdrr_source %zu\n", sizeof(gdrr_source));
    printf("gdrr_geometry %zu\n", sizeof(gdrr_geometry));
    printf("gdrr_job %zu\n", sizeof(gdrr_job));
    printf("gdrr_tuning %zu\n", sizeof(gdrr_tuning));
    printf("GDRR_STATIC_SCRATCH_BYTES %zu\n", (size_t)GDRR_STATIC_SCRATCH_BYTES);
    F(gdrr_volume, density) F(gdrr_volume, material) F(gdrr_volume, macro) F(gdrr_volume, macro_margin)
    F(gdrr_volume, macro_rho_min)
    F(gdrr_physics, mu_mass) F(gdrr_physics, response) F(gdrr_physics, rayleigh_x0_invA) F(gdrr_physics, e_cut_kev)
    F(gdrr_source, spec_e_kev) F(gdrr_source, fu) F(gdrr_source, fluence) F(gdrr_source, spec_rows)
    F(gdrr_job, geom) F(gdrr_job, n_photons) F(gdrr_job, job_id) F(gdrr_job, first_photon) F(gdrr_job, tally_offset)
    F(gdrr_tuning, defer) F(gdrr_tuning, coll_defer)
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layout_matches_binding(abi, tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(LAYOUT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    m = {"gdrr_volume": abi.Volume, "gdrr_physics": abi.Physics, "gdrr_source": abi.Source,
         "gdrr_geometry": abi.Geometry, "gdrr_job": abi.Job, "gdrr_tuning": abi.Tuning}
    assert int(got.pop("GDRR_STATIC_SCRATCH_BYTES")) == abi.STATIC_SCRATCH_BYTES
    for k, v in got.items():
        if "." in k:
            t, f = k.split(".")
            assert getattr(m[t], f).offset == int(v), k
        else:
            assert C.sizeof(m[k]) == int(v), k


def _valid_structs(abi):
    # non-null dummy device pointers: never dereferenced, the checks fail first
    p = 0x1000
    vol = abi.Volume(8, 8, 8, 2.0, 2.0, 2.0, p, p, 0, 0.0)
    phys = abi.Physics(2, 299, 1.0, 0.5, p, None, 0.35, 1.0)
    src = abi.Source(1, p, p, 16, 12, p)
    geom = abi.Geometry(1000.0, 500.0, 0.0, 0.0, 16, 12, 8.0, 8.0)
    return vol, phys, src, geom


def _call(abi, vol, phys, src, geom, n=1000, ws_bytes=1 << 30, tally=0x2000):
    L = abi.lib()
    return L.gdrr_mc_project(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom), None, 1, n, 0, 1,
                             tally, 0x3000, ws_bytes, None)


@pytest.mark.parametrize("breaker,needle", [
    (lambda v, p, s, g: setattr(v, "nx", 0), "dimensions"),
    (lambda v, p, s, g: setattr(v, "dx_mm", -1.0), "voxel sizes"),
    (lambda v, p, s, g: setattr(v, "density", None), "pointer"),
    (lambda v, p, s, g: setattr(v, "macro", 257), "macro"),
    (lambda v, p, s, g: (setattr(v, "macro", 2), setattr(v, "macro_margin", -1.0)), "macro_margin"),
    (lambda v, p, s, g: setattr(p, "n_mat", 17), "n_mat"),
    (lambda v, p, s, g: setattr(p, "n_e", 1), "n_e"),
    (lambda v, p, s, g: setattr(p, "e_cut_kev", 0.5), "e_cut"),
    (lambda v, p, s, g: setattr(s, "n_spec", 0), "n_spec"),
    (lambda v, p, s, g: setattr(s, "fu", 15), "fluence grid"),
    (lambda v, p, s, g: setattr(s, "spec_rows", 15), "spec_rows"),
    (lambda v, p, s, g: setattr(s, "spec_rows", -1), "spec_rows"),
    (lambda v, p, s, g: (setattr(s, "n_spec", 4096), setattr(s, "spec_rows", 4097), setattr(s, "fu", 4097),
                         setattr(s, "fv", 1), setattr(g, "nu", 4097), setattr(g, "nv", 1)), "2^24"),
    (lambda v, p, s, g: setattr(g, "aid_mm", 5.0), "between the source and the detector"),
    (lambda v, p, s, g: setattr(g, "du_mm", 0.0), "detector grid"),
    # 1024 x 1024 x 2047 voxels (< 2^31) but 1025 x 1025 x 2048 cells (> 2^31): 32-bit cell indices would wrap
    (lambda v, p, s, g: (setattr(v, "nx", 1024), setattr(v, "ny", 1024), setattr(v, "nz", 2047),
                         setattr(v, "dx_mm", 0.01), setattr(v, "dy_mm", 0.01), setattr(v, "dz_mm", 0.01)),
     "interpolation cells"),
])
def test_invalid_arguments_are_rejected(abi, breaker, needle):
    vol, phys, src, geom = _valid_structs(abi)
    breaker(vol, phys, src, geom)
    rc = _call(abi, vol, phys, src, geom)
    assert rc == abi.GDRR_EINVAL
    assert needle in abi.lib().gdrr_last_error().decode()


def test_too_many_photons_and_small_workspace(abi):
    vol, phys, src, geom = _valid_structs(abi)
    assert _call(abi, vol, phys, src, geom, n=(1 << 32) + 1) == abi.GDRR_EINVAL
    assert "2^32" in abi.lib().gdrr_last_error().decode()
    assert _call(abi, vol, phys, src, geom, ws_bytes=16) == abi.GDRR_EINVAL
    assert "workspace" in abi.lib().gdrr_last_error().decode()
    assert _call(abi, vol, phys, src, geom, tally=None) == abi.GDRR_EINVAL


def test_static_entry_point_rejects_before_any_device_work(abi):
    """gdrr_mc_project_static: invalid arguments, GDRR_RESUME and calls whose
    workspace exceeds the static scratch are refused on the host (the dummy
    pointers would fault if anything were launched)."""
    L = abi.lib()
    msg = lambda: L.gdrr_last_error().decode()
    call = lambda vol, phys, src, geom, flags=1, tally=0x2000: L.gdrr_mc_project_static(
        C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom), None, 1, 1000, 0, flags, tally, None)
    vol, phys, src, geom = _valid_structs(abi)
    assert call(vol, phys, src, geom, tally=None) == abi.GDRR_EINVAL and "tally" in msg()
    assert call(vol, phys, src, geom, flags=1 | abi.RESUME) == abi.GDRR_EINVAL and "RESUME" in msg()
    vol.nx = 0
    assert call(vol, phys, src, geom) == abi.GDRR_EINVAL and "dimensions" in msg()
    # 170^3 voxels: 171^3 32-byte cell records alone exceed 128 MiB
    vol, phys, src, geom = _valid_structs(abi)
    vol.nx = vol.ny = vol.nz = 170
    vol.dx_mm = vol.dy_mm = vol.dz_mm = 1.0
    need = L.gdrr_mc_project_workspace(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom))
    assert need > abi.STATIC_SCRATCH_BYTES
    assert call(vol, phys, src, geom) == abi.GDRR_EINVAL and "static scratch" in msg()


def test_workspace_query_is_positive(abi):
    vol, phys, src, geom = _valid_structs(abi)
    L = abi.lib()
    n = L.gdrr_mc_project_workspace(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom))
    assert n > 8 * 4 * 16 * 12 + 32 * 9 * 9 * 9      # tallies and a 32-byte record per lattice cell
    assert L.gdrr_majorant_workspace() >= 2048
    # a joint source (one spectrum per column) needs a CDF per row; a bad row count sizes nothing
    src.n_spec = 64
    n1 = L.gdrr_mc_project_workspace(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom))
    src.spec_rows = 16
    n2 = L.gdrr_mc_project_workspace(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom))
    assert n2 >= n1 + 15 * 64 * 8
    src.spec_rows = 7
    assert L.gdrr_mc_project_workspace(C.byref(vol), C.byref(phys), C.byref(src), C.byref(geom)) == 0
    assert L.gdrr_version().decode().startswith("gdrr")


def test_product_path_does_not_import_the_oracle():
    """The package never reaches the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1204_6367_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "gdrr_oracle" not in text and "liboracle" not in text, f


def _call_primary(abi, vol, phys, src, geom, flags=1, step=0.0, ws_bytes=1 << 30, out=0x2000):
    L = abi.lib()
    job = abi.Job()
    job.volume, job.source, job.geom = 0, 0, geom
    return L.gdrr_primary(C.byref(vol), 1, C.byref(phys), C.byref(src), 1, C.byref(job), 1, step, flags, out,
                          0x3000, ws_bytes, None)


def test_primary_rejects_bad_arguments_on_the_host(abi):
    vol, phys, src, geom = _valid_structs(abi)
    msg = lambda: abi.lib().gdrr_last_error().decode()
    assert _call_primary(abi, vol, phys, src, geom, flags=2) == abi.GDRR_EINVAL and "only" in msg()
    assert _call_primary(abi, vol, phys, src, geom, step=1e-6) == abi.GDRR_EINVAL and "2^20" in msg()
    assert _call_primary(abi, vol, phys, src, geom, step=float("nan")) == abi.GDRR_EINVAL
    assert _call_primary(abi, vol, phys, src, geom, ws_bytes=16) == abi.GDRR_EINVAL and "workspace" in msg()
    assert _call_primary(abi, vol, phys, src, geom, out=None) == abi.GDRR_EINVAL
    bad = abi.Source(1, 0x1000, 0x1000, 15, 12, 0x1000)
    assert _call_primary(abi, vol, phys, bad, geom) == abi.GDRR_EINVAL and "fluence grid" in msg()
    job = abi.Job()
    job.volume, job.source, job.geom = 0, 0, geom
    n = abi.lib().gdrr_primary_workspace(C.byref(vol), 1, C.byref(phys), C.byref(src), 1, C.byref(job), 1)
    assert n > 32 * 9 * 9 * 9                # a 32-byte record per lattice cell


def test_denoise_and_noise_reject_bad_arguments_on_the_host(abi):
    L = abi.lib()
    msg = lambda: L.gdrr_last_error().decode()
    ws = L.gdrr_denoise_workspace(3, 20, 30)
    assert ws >= 2 * 3 * 20 * 30 * 4
    dn = lambda shat=0x10000, stride=0, n=3, beta=1.0, omega=0.8, it=10, fl=1e-6, out=0x100000, wsb=ws: \
        L.gdrr_denoise(shat, stride, n, 20, 30, beta, omega, it, fl, out, 0x3000, wsb, None)
    assert dn(beta=0.0) == abi.GDRR_EINVAL and "beta" in msg()
    assert dn(omega=2.5) == abi.GDRR_EINVAL and "omega" in msg()
    assert dn(it=-1) == abi.GDRR_EINVAL
    assert dn(fl=0.0) == abi.GDRR_EINVAL and "s_floor" in msg()
    assert dn(stride=100) == abi.GDRR_EINVAL and "stride" in msg()
    assert dn(out=0x10000 + 8) == abi.GDRR_EINVAL and "overlap" in msg()
    assert dn(wsb=16) == abi.GDRR_EINVAL and "workspace" in msg()
    assert dn(shat=None) == abi.GDRR_EINVAL
    nz = lambda n=2, npix=100, ps=0, alpha=1.0: L.gdrr_noise(n, npix, 0x1000, ps, 0x2000, 0x3000, 0, 0x4000, alpha,
                                                             0x5000, None, None)
    assert nz(npix=0) == abi.GDRR_EINVAL
    assert nz(ps=50) == abi.GDRR_EINVAL and "stride" in msg()
    assert nz(alpha=float("inf")) == abi.GDRR_EINVAL


def _batch_structs(abi, first=0, n=1000):
    vol, phys, src, geom = _valid_structs(abi)
    job = abi.Job()
    job.volume, job.source, job.geom, job.n_photons, job.job_id, job.first_photon = 0, 0, geom, n, 0, first
    return vol, phys, src, job


def test_photon_index_range_is_checked(abi):
    """first_photon + n_photons must stay below 2^32 (the Philox counter word)."""
    L = abi.lib()
    vol, phys, src, job = _batch_structs(abi, first=(1 << 32) - 1000, n=1000)
    rc = L.gdrr_mc_project_batch(C.byref(vol), 1, C.byref(phys), C.byref(src), 1, C.byref(job), 1, None, 1, 1,
                                 None, 0x2000, 0x3000, 1 << 30, None)
    assert rc == abi.GDRR_EINVAL and "2^32" in L.gdrr_last_error().decode()


def test_backward_checks_every_argument_before_touching_the_gradient(abi):
    """NULL arrays and bad indices are rejected on the host; nothing is launched
    (the gradient pointer is a dummy that a launch would fault on)."""
    L = abi.lib()
    vol, phys, src, job = _batch_structs(abi)
    msg = lambda: L.gdrr_last_error().decode()
    call = lambda vols, nv=1, srcs=None, jobs=None, volume=0, maj=0x4000, adj=0x5000, grad=0x6000: \
        L.gdrr_mc_backward(vols, nv, C.byref(phys), srcs if srcs is not None else C.byref(src), 1,
                           jobs if jobs is not None else C.byref(job), 1, volume, maj, 1, 1, None, adj, grad,
                           0x3000, 1 << 30, None)
    assert call(None) == abi.GDRR_EINVAL and "NULL" in msg()
    assert call(C.byref(vol), volume=1) == abi.GDRR_EINVAL and "volume" in msg()
    assert call(C.byref(vol), maj=None) == abi.GDRR_EINVAL and "majorants" in msg()
    assert call(C.byref(vol), grad=None) == abi.GDRR_EINVAL
    bad = abi.Volume(8, 8, 0, 2.0, 2.0, 2.0, 0x1000, 0x1000, 0, 0.0)
    assert call(C.byref(bad)) == abi.GDRR_EINVAL and "dimensions" in msg()
    for floor in (-0.01, float("nan"), float("inf")):
        bad = abi.Volume(8, 8, 8, 2.0, 2.0, 2.0, 0x1000, 0x1000, 4, 0.1, floor)
        assert call(C.byref(bad)) == abi.GDRR_EINVAL and "macro_rho_min" in msg()


def test_noise_scale_in_the_library(abi):
    """alpha = sqrt(n_sim / (zeta I)) (Sec. 2.6), with the paper's calibration
    numbers: k = sqrt(n_sim / zeta) = 0.3074 for n_sim = 5e8, zeta = 5.2913e9."""
    L = abi.lib()
    a = C.c_double(0.0)
    assert L.gdrr_noise_scale(5e8, 5.2913e9, 1.0, C.byref(a)) == abi.GDRR_OK
    assert abs(a.value - 0.3074) < 5e-4
    assert L.gdrr_noise_scale(5e8, 5.2913e9, 4.0, C.byref(a)) == abi.GDRR_OK
    assert abs(a.value - 0.3074 / 2) < 3e-4
    for bad in ((0.0, 1.0, 1.0), (1.0, -1.0, 1.0), (1.0, 1.0, float("nan")), (float("inf"), 1.0, 1.0)):
        assert L.gdrr_noise_scale(*bad, C.byref(a)) == abi.GDRR_EINVAL
    assert L.gdrr_noise_scale(1.0, 1.0, 1.0, None) == abi.GDRR_EINVAL
    assert L.gdrr_input_status(None, None) == abi.GDRR_EINVAL
