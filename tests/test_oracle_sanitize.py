"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
code only) runs every entry point on small inputs without a report: out-of-
bounds reads or writes, use after free, signed overflow, misaligned or
out-of-range conversions abort the child process.  CPU only."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import numpy as np
    import oracle
    from paper_1204_6367_amd import workloads as W

    assert oracle._LIB.endswith("liboracle_asan.so"), oracle._LIB
    ph = W.ellipsoid_phantom((10, 12, 14), (6.0, 6.0, 6.0), 5, n_inner=4)
    geom = W.Geometry(phi_rad=0.7, nu=20, nv=14, du_mm=9.0, dv_mm=9.0)
    prob = W.Problem(ph, W.physics_for(ph), W.pelvis_source(geom), geom, 0)
    p = oracle.Problem.from_workload(prob)
    mb = oracle.majorant(p, True, margin=0.1)
    oracle.majorant(p, False)
    for interp in (True, False):
        for mode in (0, 1, 2):
            oracle.mc_project(p, 3, 3000, job_id=2, interp=interp, mode=mode, trace=True, nthreads=2)
    oracle.mc_histories(p, 3, np.arange(0, 400, 3), mb, job_id=2, nthreads=2)
    adj = np.ones((2, geom.nv, geom.nu))
    oracle.mc_backward(p, 3, 3000, adj, mb, job_id=2, nthreads=2)
    oracle.mc_backward(p, 3, 3000, adj, mb, job_id=2, interp=False, nthreads=2)
    pl = oracle.Problem.from_workload(prob).local_majorants(3, 0.1)
    oracle.mc_project(pl, 3, 3000, trace=True, nthreads=2)
    oracle.mc_backward(pl, 3, 3000, adj, None, nthreads=2)
    xyz = np.random.default_rng(0).uniform(-40, 40, (200, 3))
    oracle.local_majorant_at(pl, xyz, np.full(200, 60.0))
    oracle.density_at(p, xyz, True)
    oracle.rho_integrals(p, [-50.0, -3.0, 1.0], [40.0, 7.0, -2.0])
    oracle.rho_integrals_many(p, [-50.0, -3.0, 1.0], xyz[:20])
    oracle.primary_exact(p, True, 2)
    oracle.primary_raytrace(p, True)
    oracle.primary_raytrace(p, False, pixels=[0, 5, geom.nu * geom.nv - 1])
    js = W.pelvis_source(geom, joint=True)
    pj = oracle.Problem.from_workload(W.Problem(ph, W.physics_for(ph), js, geom, 0))
    oracle.mc_project(pj, 4, 2000, trace=True, nthreads=2)
    oracle.primary_raytrace(pj, True)
    img = np.abs(np.random.default_rng(1).normal(1.0, 0.3, (3, 7, 9)))
    oracle.denoise(img, 2.0, 5)
    oracle.noise(img, img * 0.9, img, img * 1.1, 0.3)
    oracle.noise_scale(5e8, 5.2913e9, 0.6)
    oracle.sample_compton(60.0, 1, 1000)
    oracle.sample_rayleigh(30.0, 0.35, 1, 1000)
    oracle.rotate([0.0, 0.0, 1.0], 0.3, 0.2)
    oracle.geometry(p)
    oracle.philox([1, 2, 3, 4], [5, 6])
    print("SANITIZED_OK")
""")


def test_oracle_under_asan_ubsan(tmp_path):
    import oracle
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not libasan or not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = oracle.build(force=True, out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    env = dict(os.environ)
    env.update(GDRR_ORACLE_LIB=lib, LD_PRELOAD=libasan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=600,
                       cwd=str(tmp_path))
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
