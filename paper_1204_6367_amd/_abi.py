"""ctypes mirror of include/gdrr.h and the loader of libgdrr.so.

Argument marshalling only: every step of the projection runs in the HIP
library.  There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgdrr.so")

GDRR_OK = 0
GDRR_EINVAL = -1
GDRR_EHIP = -2
GDRR_ENOTSUP = -3

INTERP_DENSITY = 1
TALLY_SUMSQ = 2
ACCUMULATE = 4
SCATTER_FIRST = 8
SCATTER_FIRST_COMPTON = 16
RESUME = 32

STATIC_SCRATCH_BYTES = 128 << 20     # the per-device scratch of gdrr_mc_project_static

MAX_MATERIALS = 16
MAX_VOLUMES = 8
MAX_SOURCES = 8


class Volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx_mm", C.c_float), ("dy_mm", C.c_float), ("dz_mm", C.c_float),
                ("density", C.c_void_p), ("material", C.c_void_p),
                ("macro", C.c_int32), ("macro_margin", C.c_float), ("macro_rho_min", C.c_float)]


class Physics(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("n_e", C.c_int32),
                ("e0_kev", C.c_float), ("de_kev", C.c_float),
                ("mu_mass", C.c_void_p), ("response", C.c_void_p),
                ("rayleigh_x0_invA", C.c_float), ("e_cut_kev", C.c_float)]


class Source(C.Structure):
    _fields_ = [("n_spec", C.c_int32), ("spec_e_kev", C.c_void_p), ("spec_prob", C.c_void_p),
                ("fu", C.c_int32), ("fv", C.c_int32), ("fluence", C.c_void_p), ("spec_rows", C.c_int32)]


class Geometry(C.Structure):
    _fields_ = [("sad_mm", C.c_float), ("aid_mm", C.c_float),
                ("phi_rad", C.c_float), ("theta_rad", C.c_float),
                ("nu", C.c_int32), ("nv", C.c_int32),
                ("du_mm", C.c_float), ("dv_mm", C.c_float)]


class Job(C.Structure):
    _fields_ = [("volume", C.c_int32), ("source", C.c_int32), ("geom", Geometry),
                ("n_photons", C.c_uint64), ("job_id", C.c_uint32), ("first_photon", C.c_uint32),
                ("tally_offset", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("chunk", C.c_int32), ("defer", C.c_int32), ("coll_defer", C.c_int32)]


# every function the header declares, with its ctypes signature
_P, _vp, _sz = C.POINTER, C.c_void_p, C.c_size_t
SIGNATURES = {
    "gdrr_majorant": (C.c_int, [_P(Volume), _P(Physics), C.c_uint32, C.c_float, _vp, _vp, _sz, _vp]),
    "gdrr_majorant_workspace": (_sz, []),
    "gdrr_mc_project": (C.c_int, [_P(Volume), _P(Physics), _P(Source), _P(Geometry), _vp, C.c_uint64,
                                  C.c_uint64, C.c_uint32, C.c_uint32, _vp, _vp, _sz, _vp]),
    "gdrr_mc_project_workspace": (_sz, [_P(Volume), _P(Physics), _P(Source), _P(Geometry)]),
    "gdrr_mc_project_static": (C.c_int, [_P(Volume), _P(Physics), _P(Source), _P(Geometry), _vp, C.c_uint64,
                                         C.c_uint64, C.c_uint32, C.c_uint32, _vp, _vp]),
    "gdrr_mc_project_batch": (C.c_int, [_P(Volume), C.c_int32, _P(Physics), _P(Source), C.c_int32, _P(Job),
                                        C.c_int32, _vp, C.c_uint64, C.c_uint32, _P(Tuning), _vp, _vp, _sz,
                                        _vp]),
    "gdrr_mc_project_batch_workspace": (_sz, [_P(Volume), C.c_int32, _P(Physics), _P(Source), C.c_int32,
                                             _P(Job), C.c_int32]),
    "gdrr_mc_backward": (C.c_int, [_P(Volume), C.c_int32, _P(Physics), _P(Source), C.c_int32, _P(Job),
                                   C.c_int32, C.c_int32, _vp, C.c_uint64, C.c_uint32, _P(Tuning), _vp, _vp,
                                   _vp, _sz, _vp]),
    "gdrr_mc_trace": (C.c_int, [_P(Volume), _P(Physics), _P(Source), _P(Geometry), _vp, C.c_uint64,
                                C.c_uint64, C.c_uint32, C.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                _vp]),
    "gdrr_primary": (C.c_int, [_P(Volume), C.c_int32, _P(Physics), _P(Source), C.c_int32, _P(Job), C.c_int32,
                               C.c_float, C.c_uint32, _vp, _vp, _sz, _vp]),
    "gdrr_primary_workspace": (_sz, [_P(Volume), C.c_int32, _P(Physics), _P(Source), C.c_int32, _P(Job),
                                     C.c_int32]),
    "gdrr_denoise": (C.c_int, [_vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_int32,
                               C.c_float, _vp, _vp, _sz, _vp]),
    "gdrr_denoise_workspace": (_sz, [C.c_int32, C.c_int32, C.c_int32]),
    "gdrr_noise": (C.c_int, [C.c_int32, C.c_int64, _vp, C.c_int64, _vp, _vp, C.c_int64, _vp, C.c_double, _vp, _vp,
                             _vp]),
    "gdrr_noise_scale": (C.c_int, [C.c_double, C.c_double, C.c_double, _P(C.c_double)]),
    "gdrr_input_status": (C.c_int, [_vp, _vp]),
    "gdrr_enable_timing": (C.c_int, [C.c_int]),
    "gdrr_last_kernel_ms": (C.c_int, [_P(C.c_float)]),
    "gdrr_default_tuning": (C.c_int, [_P(Tuning)]),
    "gdrr_init": (C.c_int, []),
    "gdrr_last_error": (C.c_char_p, []),
    "gdrr_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load libgdrr.so (built by paper_1204_6367_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1204_6367_amd.build` "
                              "(the projection has no other implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class GdrrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gdrr error {code}: {msg}")
        self.code = code


def check(rc: int):
    if rc != GDRR_OK:
        raise GdrrError(rc, lib().gdrr_last_error().decode(errors="replace"))
