"""CPU oracle for the gDRR Monte Carlo projection step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It wraps `gdrr_oracle.c` (plain double-precision C, see its header)
through ctypes.  It never imports the GPU package, and the GPU package never
imports it; both receive the arrays made by the seeded input generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gdrr_oracle.c")
# GDRR_ORACLE_LIB points the loader at another build of the same source (the
# sanitizer build of the CPU tests)
_LIB = os.environ.get("GDRR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CLASS_NAMES = ["primary", "scatter", "absorbed", "cut", "missed", "lost"]


SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                  "-g"]


def build(force: bool = True, out: Optional[str] = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math).
    sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build (host
    code only) at `out`, for the CPU tests."""
    lib_path = out or _LIB
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC):
        tmp = lib_path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
               *(SANITIZE_FLAGS if sanitize else []), _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return lib_path


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("density", C.c_void_p), ("material", C.c_void_p),
        ("n_mat", C.c_int32), ("n_e", C.c_int32),
        ("e0", C.c_double), ("de", C.c_double),
        ("mu", C.c_void_p), ("response", C.c_void_p),
        ("x0_rayleigh", C.c_double), ("e_cut", C.c_double),
        ("n_spec", C.c_int32),
        ("spec_e", C.c_void_p), ("spec_p", C.c_void_p), ("spec_rows", C.c_int32), ("fluence", C.c_void_p),
        ("sad", C.c_double), ("aid", C.c_double), ("phi", C.c_double), ("theta", C.c_double),
        ("nu", C.c_int32), ("nv", C.c_int32),
        ("du", C.c_double), ("dv", C.c_double),
        ("macro", C.c_int32), ("macro_margin", C.c_double), ("macro_rho_min", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        vp, u64, i32 = C.c_void_p, C.c_uint64, C.c_int32
        L.or_philox.argtypes = [vp, vp, vp]
        L.or_philox.restype = None
        L.or_majorant.argtypes = [P, i32, vp]
        L.or_majorant_margin.argtypes = [P, i32, C.c_double, vp]
        L.or_mc_project.argtypes = [P, u64, u64, C.c_uint32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32]
        L.or_mc_backward.argtypes = [P, u64, u64, C.c_uint32, i32, i32, vp, vp, vp, i32]
        L.or_rho_integrals.argtypes = [P, i32, vp, vp, vp]
        L.or_mc_histories.argtypes = [P, u64, C.c_uint32, i32, vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp, i32]
        L.or_primary_exact.argtypes = [P, i32, i32, vp]
        L.or_primary_raytrace.argtypes = [P, i32, C.c_double, vp, C.c_int64, vp]
        L.or_denoise.argtypes = [vp, vp, i32, i32, i32, C.c_double, C.c_double, i32, C.c_double, vp]
        L.or_noise.argtypes = [C.c_int64, vp, vp, vp, vp, C.c_double, vp, vp]
        L.or_noise_scale.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_local_majorant_at.argtypes = [P, vp, vp, C.c_int64, vp]
        L.or_noise_scale.restype = C.c_double
        L.or_rho_integrals_many.argtypes = [P, i32, vp, vp, C.c_int64, vp]
        L.or_sample_compton.argtypes = [C.c_double, u64, u64, vp, vp]
        L.or_sample_rayleigh.argtypes = [C.c_double, C.c_double, u64, u64, vp]
        L.or_rotate.argtypes = [vp, C.c_double, C.c_double, vp]
        L.or_rotate.restype = None
        L.or_geometry.argtypes = [P, vp]
        L.or_geometry.restype = None
        L.or_density_at.argtypes = [P, i32, vp, C.c_int64, vp]
        L.or_sample_cdf.argtypes = [vp, i32, vp, C.c_int64, vp]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Problem:
    """Holds contiguous copies of the inputs and the ctypes struct over them.

    Arguments mirror the generator's dataclasses but are taken field by field
    so that this package does not import the GPU package."""

    def __init__(self, density, material, spacing_mm, mu_mass, e0_kev, de_kev,
                 spec_e, spec_p, fluence, sad_mm, aid_mm, phi_rad, theta_rad,
                 nu, nv, du_mm, dv_mm, response=None, x0_rayleigh=0.35, e_cut_kev=1.0):
        self.density = np.ascontiguousarray(density, np.float32)
        self.material = np.ascontiguousarray(material, np.uint8)
        self.mu = np.ascontiguousarray(mu_mass, np.float32)
        self.spec_e = np.ascontiguousarray(spec_e, np.float32)
        self.spec_p = np.ascontiguousarray(spec_p, np.float32)
        self.fluence = np.ascontiguousarray(fluence, np.float32)
        self.response = None if response is None else np.ascontiguousarray(response, np.float32)
        nz, ny, nx = self.density.shape
        self.nu, self.nv = int(nu), int(nv)
        self.shape = (nz, ny, nx)
        s = _Problem()
        s.nx, s.ny, s.nz = nx, ny, nz
        s.dx, s.dy, s.dz = map(float, spacing_mm)
        s.density, s.material = _ptr(self.density), _ptr(self.material)
        s.n_mat, s.n_e = self.mu.shape[0], self.mu.shape[1]
        s.e0, s.de = float(e0_kev), float(de_kev)
        s.mu, s.response = _ptr(self.mu), _ptr(self.response)
        s.x0_rayleigh, s.e_cut = float(x0_rayleigh), float(e_cut_kev)
        s.n_spec = self.spec_e.shape[0]
        # a [nu][n_spec] table is the joint source phi(E|u): one spectrum per detector column
        if self.spec_p.ndim == 2:
            if self.spec_p.shape != (self.nu, s.n_spec):
                raise ValueError("a joint spectrum table must be [nu][n_spec]")
            s.spec_rows = self.nu
        elif self.spec_p.shape != (s.n_spec,):
            raise ValueError("spec_p must be [n_spec] or [nu][n_spec]")
        s.spec_e, s.spec_p, s.fluence = _ptr(self.spec_e), _ptr(self.spec_p), _ptr(self.fluence)
        s.sad, s.aid, s.phi, s.theta = float(sad_mm), float(aid_mm), float(phi_rad), float(theta_rad)
        s.nu, s.nv = self.nu, self.nv
        s.du, s.dv = float(du_mm), float(dv_mm)
        self.s = s

    @classmethod
    def from_workload(cls, prob, phi_rad=None, density=None):
        """Build from a generator `Problem` (duck-typed; no import of it)."""
        ph, phys, src, g = prob.phantom, prob.physics, prob.source, prob.geom
        return cls(ph.density if density is None else density, ph.material, ph.spacing_mm,
                   phys.mu_mass, phys.grid.e0_kev, phys.grid.de_kev, src.spec_e, src.spec_p,
                   src.fluence, g.sad_mm, g.aid_mm, g.phi_rad if phi_rad is None else phi_rad,
                   g.theta_rad, g.nu, g.nv, g.du_mm, g.dv_mm, phys.response,
                   phys.rayleigh_x0, phys.e_cut_kev)

    def local_majorants(self, macro: int, margin: float = 2.0**-20, rho_min: float = 0.0) -> "Problem":
        """Switch the transport to local majorants on cubes of macro^3 voxels (0: back to the
        global one); each cube's bound assumes a density of at least rho_min g/cm^3."""
        self.s.macro = int(macro)
        self.s.macro_margin = float(margin)
        self.s.macro_rho_min = float(rho_min)
        return self

    @property
    def ref(self):
        return C.byref(self.s)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def majorant(p: Problem, interp: bool = True, margin: float = 2.0**-20) -> np.ndarray:
    out = np.zeros(p.mu.shape[1] - 1, np.float64)
    if lib().or_majorant_margin(p.ref, int(interp), float(margin), _ptr(out)):
        raise ValueError("oracle majorant: invalid input")
    return out


def mc_project(p: Problem, seed: int, n: int, job_id: int = 0, interp: bool = True,
               mode: int = 0, majorant_tab: Optional[np.ndarray] = None, trace: bool = False,
               nthreads: int = 0):
    """Returns dict(tally=[4][nv][nu], stats=..., and per-history arrays if trace)."""
    tally = np.zeros((4, p.nv, p.nu), np.float64)
    stats = np.zeros(14, np.float64)
    tr = {}
    if trace:
        tr = dict(cls=np.zeros(n, np.int8), pixel=np.zeros(n, np.int32),
                  e_final=np.zeros(n, np.float64), steps=np.zeros(n, np.int32),
                  n_compton=np.zeros(n, np.int32), n_rayleigh=np.zeros(n, np.int32))
    mb = None if majorant_tab is None else np.ascontiguousarray(majorant_tab, np.float64)
    rc = lib().or_mc_project(p.ref, seed, n, job_id, int(interp), mode, _ptr(mb), _ptr(tally),
                             _ptr(tr.get("cls")), _ptr(tr.get("pixel")), _ptr(tr.get("e_final")),
                             _ptr(tr.get("steps")), _ptr(tr.get("n_compton")),
                             _ptr(tr.get("n_rayleigh")), _ptr(stats), nthreads)
    if rc:
        raise ValueError("oracle mc_project: invalid input")
    out = dict(tally=tally, stats=dict(
        steps=stats[0], real=stats[1], compton=stats[2], rayleigh=stats[3],
        classes={CLASS_NAMES[k]: stats[4 + k] for k in range(6)},
        e_src=stats[10], e_out=stats[11], tries=stats[12], crossings=stats[13]))
    out.update(tr)
    return out


def mc_histories(p: Problem, seed: int, ids, majorant_tab: np.ndarray, job_id: int = 0,
                 interp: bool = True, nthreads: int = 0):
    """Outcomes of the selected photon indices (same definition as mc_project's trace)."""
    ids = np.ascontiguousarray(ids, np.uint32)
    m = ids.shape[0]
    tr = dict(cls=np.zeros(m, np.int8), pixel=np.zeros(m, np.int32), e_final=np.zeros(m, np.float64),
              steps=np.zeros(m, np.int32), n_compton=np.zeros(m, np.int32), n_rayleigh=np.zeros(m, np.int32))
    mb = None if majorant_tab is None else np.ascontiguousarray(majorant_tab, np.float64)
    rc = lib().or_mc_histories(p.ref, seed, job_id, int(interp), _ptr(mb), _ptr(ids), m, _ptr(tr["cls"]),
                               _ptr(tr["pixel"]), _ptr(tr["e_final"]), _ptr(tr["steps"]),
                               _ptr(tr["n_compton"]), _ptr(tr["n_rayleigh"]), nthreads)
    if rc:
        raise ValueError("oracle mc_histories: invalid input")
    return tr


def mc_backward(p: Problem, seed: int, n: int, adj: np.ndarray, majorant_tab: np.ndarray,
                job_id: int = 0, interp: bool = True, mode: int = 0, grad: Optional[np.ndarray] = None,
                nthreads: int = 0) -> np.ndarray:
    adj = np.ascontiguousarray(adj, np.float64)
    assert adj.shape == (2, p.nv, p.nu)
    if grad is None:
        grad = np.zeros(p.shape, np.float64)
    mb = None if majorant_tab is None else np.ascontiguousarray(majorant_tab, np.float64)
    if lib().or_mc_backward(p.ref, seed, n, job_id, int(interp), mode, _ptr(mb), _ptr(adj), _ptr(grad), nthreads):
        raise ValueError("oracle mc_backward: invalid input")
    return grad


def rho_integrals(p: Problem, a, b, interp: bool = True) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    out = np.zeros(p.mu.shape[0], np.float64)
    lib().or_rho_integrals(p.ref, int(interp), _ptr(a), _ptr(b), _ptr(out))
    return out


def rho_integrals_many(p: Problem, a, b, interp: bool = True) -> np.ndarray:
    """Segments a -> b[k]: [m][n_mat] integrals of rho over each material."""
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64).reshape(-1, 3)
    out = np.zeros((b.shape[0], p.mu.shape[0]), np.float64)
    if lib().or_rho_integrals_many(p.ref, int(interp), _ptr(a), _ptr(b), b.shape[0], _ptr(out)):
        raise ValueError("oracle rho_integrals_many failed")
    return out


def primary_exact(p: Problem, interp: bool = True, nq: int = 8) -> np.ndarray:
    out = np.zeros((p.nv, p.nu), np.float64)
    if lib().or_primary_exact(p.ref, int(interp), nq, _ptr(out)):
        raise ValueError("oracle primary_exact: invalid input")
    return out


def primary_raytrace(p: Problem, interp: bool = True, dl: float = 0.0, pixels=None) -> np.ndarray:
    """Eq. 1 by ray tracing (Sec. 2.3): per pixel, per source photon.  `dl` in
    mm (<= 0: half the smallest voxel edge).  `pixels`: flat indices iv*nu+iu
    (returns [m]), or None for the whole detector ([nv][nu])."""
    if pixels is None:
        out = np.zeros((p.nv, p.nu), np.float64)
        rc = lib().or_primary_raytrace(p.ref, int(interp), float(dl), None, 0, _ptr(out))
    else:
        px = np.ascontiguousarray(pixels, np.int32).ravel()
        out = np.zeros(px.size, np.float64)
        rc = lib().or_primary_raytrace(p.ref, int(interp), float(dl), _ptr(px), px.size, _ptr(out))
    if rc:
        raise ValueError("oracle primary_raytrace: invalid input")
    return out


def denoise(shat, beta: float, iters: int, omega: float = 0.8, s_floor: float = 1e-12, s0=None) -> np.ndarray:
    """Eq. 5 (Sec. 2.5) on [nv][nu] or [n][nv][nu] images; S^(0) = Shat unless s0 is given."""
    h = np.ascontiguousarray(shat, np.float64)
    shape = h.shape
    h3 = h.reshape((-1,) + shape[-2:])
    g = None if s0 is None else np.ascontiguousarray(s0, np.float64).reshape(h3.shape)
    out = np.zeros_like(h3)
    if lib().or_denoise(_ptr(h3), _ptr(g), h3.shape[0], h3.shape[1], h3.shape[2], float(beta), float(omega),
                        int(iters), float(s_floor), _ptr(out)):
        raise ValueError("oracle denoise: invalid input")
    return out.reshape(shape)


def local_majorant_at(p: Problem, xyz, e) -> np.ndarray:
    """Local majorant (1/cm) of the cube holding each position at each energy."""
    x = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    ee = np.ascontiguousarray(e, np.float64).ravel()
    out = np.zeros(len(ee), np.float64)
    if lib().or_local_majorant_at(p.ref, _ptr(x), _ptr(ee), len(ee), _ptr(out)):
        raise ValueError("oracle local_majorant_at: invalid input")
    return out


def noise_scale(n_sim: float, zeta: float, mas: float) -> float:
    a = lib().or_noise_scale(float(n_sim), float(zeta), float(mas))
    if a < 0:
        raise ValueError("oracle noise_scale: invalid input")
    return a


def noise(phat, p, shat, s, alpha: float):
    """Sec. 2.6: (N, P + S + N) with N = alpha ((Phat - P) + (Shat - S))."""
    arrs = [np.ascontiguousarray(x, np.float64) for x in (phat, p, shat, s)]
    n_out = np.zeros_like(arrs[0])
    img = np.zeros_like(arrs[0])
    if lib().or_noise(arrs[0].size, *map(_ptr, arrs), float(alpha), _ptr(n_out), _ptr(img)):
        raise ValueError("oracle noise: invalid input")
    return n_out, img


def sample_compton(e_kev: float, seed: int, n: int):
    cost = np.zeros(n, np.float64)
    tau = np.zeros(n, np.float64)
    lib().or_sample_compton(e_kev, seed, n, _ptr(cost), _ptr(tau))
    return cost, tau


def sample_rayleigh(e_kev: float, x0: float, seed: int, n: int) -> np.ndarray:
    cost = np.zeros(n, np.float64)
    lib().or_sample_rayleigh(e_kev, x0, seed, n, _ptr(cost))
    return cost


def rotate(d, cost: float, phi: float) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(3, np.float64)
    lib().or_rotate(_ptr(d), cost, phi, _ptr(out))
    return out


def geometry(p: Problem):
    out = np.zeros(15, np.float64)
    lib().or_geometry(p.ref, _ptr(out))
    return dict(S=out[0:3], P=out[3:6], n=out[6:9], eu=out[9:12], ev=out[12:15])


def density_at(p: Problem, xyz, interp: bool = True) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    out = np.zeros(xyz.shape[0], np.float64)
    lib().or_density_at(p.ref, int(interp), _ptr(xyz), xyz.shape[0], _ptr(out))
    return out


def sample_cdf(w, u) -> np.ndarray:
    w = np.ascontiguousarray(w, np.float32)
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros(u.shape[0], np.int32)
    if lib().or_sample_cdf(_ptr(w), w.shape[0], _ptr(u), u.shape[0], _ptr(out)):
        raise ValueError("invalid weights")
    return out
