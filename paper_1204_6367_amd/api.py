"""Python binding of libgdrr: device containers for the inputs, thin
wrappers over the C ABI, and the autograd Function.

PyTorch provides device memory and the stream; every step of the projection
(majorant, source tables, transport, scoring, finalisation, adjoint) runs in
the HIP library.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi

INTERP_DENSITY = _abi.INTERP_DENSITY
TALLY_SUMSQ = _abi.TALLY_SUMSQ
ACCUMULATE = _abi.ACCUMULATE
SCATTER_FIRST = _abi.SCATTER_FIRST
SCATTER_FIRST_COMPTON = _abi.SCATTER_FIRST_COMPTON
RESUME = _abi.RESUME


def _dev(device):
    return torch.device(device if device is not None else "cuda")


def _stream(stream) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _t(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device).contiguous()


class DeviceVolume:
    """Voxel phantom on the device: density [nz][ny][nx] f32, material u8."""

    def __init__(self, density, material, spacing_mm, device=None):
        dev = _dev(device)
        self.density = _t(density, torch.float32, dev)
        self.material = _t(material, torch.uint8, dev)
        assert self.density.shape == self.material.shape and self.density.dim() == 3
        self.spacing_mm = tuple(float(s) for s in spacing_mm)
        self.macro, self.macro_margin, self.macro_rho_min = 0, 2.0**-20, 0.0

    def local_majorants(self, macro: int, margin: float = 2.0**-20, rho_min: float = 0.0) -> "DeviceVolume":
        """Track with local majorants on cubes of macro^3 voxels (0: one majorant per energy
        interval); each cube's bound assumes a density of at least rho_min g/cm^3."""
        self.macro, self.macro_margin, self.macro_rho_min = int(macro), float(margin), float(rho_min)
        return self

    @property
    def shape(self):
        return tuple(self.density.shape)

    def struct(self, density: Optional[torch.Tensor] = None) -> _abi.Volume:
        d = self.density if density is None else density
        nz, ny, nx = d.shape
        return _abi.Volume(nx, ny, nz, *self.spacing_mm, d.data_ptr(), self.material.data_ptr(), self.macro,
                           self.macro_margin, self.macro_rho_min)


class DevicePhysics:
    """Mass attenuation tables [n_mat][n_e][3] and optional response [n_e]."""

    def __init__(self, mu_mass, e0_kev, de_kev, response=None, rayleigh_x0=0.35, e_cut_kev=1.0, device=None):
        dev = _dev(device)
        self.mu = _t(mu_mass, torch.float32, dev)
        self.response = None if response is None else _t(response, torch.float32, dev)
        self.e0, self.de = float(e0_kev), float(de_kev)
        self.x0, self.e_cut = float(rayleigh_x0), float(e_cut_kev)

    @property
    def n_e(self):
        return self.mu.shape[1]

    def struct(self) -> _abi.Physics:
        return _abi.Physics(self.mu.shape[0], self.mu.shape[1], self.e0, self.de, self.mu.data_ptr(),
                            None if self.response is None else self.response.data_ptr(), self.x0, self.e_cut)


class DeviceSource:
    """Spectrum (energies, weights) and fluence map [nv][nu] weights.  Weights
    of shape [nu][n_spec] make a joint source: one spectrum per detector column."""

    def __init__(self, spec_e, spec_p, fluence, device=None):
        dev = _dev(device)
        self.spec_e = _t(spec_e, torch.float32, dev)
        self.spec_p = _t(spec_p, torch.float32, dev)
        self.fluence = _t(fluence, torch.float32, dev)
        if self.fluence.dim() != 2:
            raise ValueError("fluence must be [nv][nu]")
        n, fu = self.spec_e.shape[0], self.fluence.shape[1]
        if self.spec_p.shape not in (torch.Size([n]), torch.Size([fu, n])):
            raise ValueError("spectrum weights must be [n_spec] or [nu][n_spec]")

    def struct(self) -> _abi.Source:
        fv, fu = self.fluence.shape
        rows = fu if self.spec_p.dim() == 2 else 0
        return _abi.Source(self.spec_e.shape[0], self.spec_e.data_ptr(), self.spec_p.data_ptr(), fu, fv,
                           self.fluence.data_ptr(), rows)


def geometry_struct(g) -> _abi.Geometry:
    """From any object with sad_mm, aid_mm, phi_rad, theta_rad, nu, nv, du_mm, dv_mm."""
    return _abi.Geometry(g.sad_mm, g.aid_mm, g.phi_rad, g.theta_rad, g.nu, g.nv, g.du_mm, g.dv_mm)


def upload(problem, device=None):
    """Device copies of a workloads.Problem: (volume, physics, source)."""
    ph, phys, src = problem.phantom, problem.physics, problem.source
    vol = DeviceVolume(ph.density, ph.material, ph.spacing_mm, device)
    dphys = DevicePhysics(phys.mu_mass, phys.grid.e0_kev, phys.grid.de_kev, phys.response,
                          phys.rayleigh_x0, phys.e_cut_kev, device)
    dsrc = DeviceSource(src.spec_e, src.spec_p, src.fluence, device)
    return vol, dphys, dsrc


def _flags(interp: bool, sumsq: bool, extra: int = 0) -> int:
    return (INTERP_DENSITY if interp else 0) | (TALLY_SUMSQ if sumsq else 0) | extra


def majorant(vol: DeviceVolume, phys: DevicePhysics, interp: bool = True, margin: float = 2.0**-20,
             density: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    L = _abi.lib()
    out = torch.empty(phys.n_e - 1, dtype=torch.float32, device=vol.density.device)
    ws = torch.empty(int(L.gdrr_majorant_workspace()), dtype=torch.uint8, device=vol.density.device)
    v, p = vol.struct(density), phys.struct()
    _abi.check(L.gdrr_majorant(C.byref(v), C.byref(p), INTERP_DENSITY if interp else 0, margin,
                               out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def project(vol: DeviceVolume, phys: DevicePhysics, src: DeviceSource, geom, n_photons: int, seed: int = 1,
            job_id: int = 0, interp: bool = True, sumsq: bool = True, majorant_tab: Optional[torch.Tensor] = None,
            flags: int = 0, out: Optional[torch.Tensor] = None, density: Optional[torch.Tensor] = None,
            stream=None) -> torch.Tensor:
    """One projection: tally [4][nv][nu] float64 (P, P^2, S, S^2 per source photon)."""
    L = _abi.lib()
    g = geometry_struct(geom)
    v, p, s = vol.struct(density), phys.struct(), src.struct()
    if out is None:
        out = torch.zeros(4, geom.nv, geom.nu, dtype=torch.float64, device=vol.density.device)
    nbytes = int(L.gdrr_mc_project_workspace(C.byref(v), C.byref(p), C.byref(s), C.byref(g)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=vol.density.device)
    mb = None if majorant_tab is None else majorant_tab.data_ptr()
    _abi.check(L.gdrr_mc_project(C.byref(v), C.byref(p), C.byref(s), C.byref(g), mb, seed, n_photons, job_id,
                                 _flags(interp, sumsq, flags), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream(stream)))
    return out


def project_static(vol: DeviceVolume, phys: DevicePhysics, src: DeviceSource, geom, n_photons: int, seed: int = 1,
                   job_id: int = 0, interp: bool = True, sumsq: bool = True,
                   majorant_tab: Optional[torch.Tensor] = None, flags: int = 0,
                   out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """project() through gdrr_mc_project_static: no workspace, the library's
    per-device static scratch (calls on one device must not overlap).  With
    `out` given, nothing is allocated here either."""
    L = _abi.lib()
    g = geometry_struct(geom)
    v, p, s = vol.struct(), phys.struct(), src.struct()
    if out is None:
        out = torch.zeros(4, geom.nv, geom.nu, dtype=torch.float64, device=vol.density.device)
    mb = None if majorant_tab is None else majorant_tab.data_ptr()
    _abi.check(L.gdrr_mc_project_static(C.byref(v), C.byref(p), C.byref(s), C.byref(g), mb, seed, n_photons,
                                        job_id, _flags(interp, sumsq, flags), out.data_ptr(), _stream(stream)))
    return out


def trace(vol: DeviceVolume, phys: DevicePhysics, src: DeviceSource, geom, n_photons: int, seed: int = 1,
          job_id: int = 0, interp: bool = True, majorant_tab: Optional[torch.Tensor] = None,
          stream=None) -> Dict[str, torch.Tensor]:
    """Per-history outcomes (class, pixel, final energy, flights, Compton and Rayleigh counts)."""
    L = _abi.lib()
    dev = vol.density.device
    out = dict(cls=torch.full((n_photons,), -1, dtype=torch.int8, device=dev),
               pixel=torch.empty(n_photons, dtype=torch.int32, device=dev),
               e_final=torch.empty(n_photons, dtype=torch.float32, device=dev),
               steps=torch.empty(n_photons, dtype=torch.int32, device=dev),
               n_compton=torch.empty(n_photons, dtype=torch.int32, device=dev),
               n_rayleigh=torch.empty(n_photons, dtype=torch.int32, device=dev))
    g = geometry_struct(geom)
    v, p, s = vol.struct(), phys.struct(), src.struct()
    nbytes = int(L.gdrr_mc_project_workspace(C.byref(v), C.byref(p), C.byref(s), C.byref(g)))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    mb = None if majorant_tab is None else majorant_tab.data_ptr()
    _abi.check(L.gdrr_mc_trace(C.byref(v), C.byref(p), C.byref(s), C.byref(g), mb, seed, n_photons, job_id,
                               INTERP_DENSITY if interp else 0, out["cls"].data_ptr(), out["pixel"].data_ptr(),
                               out["e_final"].data_ptr(), out["steps"].data_ptr(), out["n_compton"].data_ptr(),
                               out["n_rayleigh"].data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def primary(vol: DeviceVolume, phys: DevicePhysics, src: DeviceSource, geom, interp: bool = True,
            step_mm: float = 0.0, density: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Eq. 1 by ray tracing: primary signal [nv][nu] float64 per source photon."""
    b = Batch([vol], phys, [src], [JobSpec(geom, 0, 0)])
    return b.primary(interp=interp, step_mm=step_mm, densities=None if density is None else [density],
                     stream=stream)[0]


def _image_stack(x: torch.Tensor, name: str):
    """(tensor, n, nv, nu, image stride) of [n][nv][nu] or [nv][nu] float64 images whose rows are contiguous."""
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dim() != 3 or x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError(f"{name}: expected float64 [n][nv][nu] or [nv][nu] on the GPU")
    n, nv, nu = x.shape
    if x.stride(2) != 1 or (nv > 1 and x.stride(1) != nu):
        raise ValueError(f"{name}: each image must be a contiguous [nv][nu] block")
    return x, n, nv, nu, x.stride(0) if n > 1 else nv * nu


def denoise(shat: torch.Tensor, beta: float, iters: int, omega: float = 0.8, s_floor: float = 1e-6,
            out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Eq. 5 (Sec. 2.5) on float64 images [n][nv][nu] (or [nv][nu]); the images may be
    strided views such as plane 2 of a batch's tallies.  Returns [n][nv][nu] float64."""
    L = _abi.lib()
    x, n, nv, nu, stride = _image_stack(shat, "shat")
    if out is None:
        out = torch.empty(n, nv, nu, dtype=torch.float64, device=x.device)
    ws = torch.empty(int(L.gdrr_denoise_workspace(n, nv, nu)), dtype=torch.uint8, device=x.device)
    _abi.check(L.gdrr_denoise(x.data_ptr(), stride, n, nv, nu, float(beta), float(omega), int(iters),
                              float(s_floor), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out if shat.dim() == 3 else out[0]


def noise(phat: torch.Tensor, p: torch.Tensor, shat: torch.Tensor, s: torch.Tensor, alpha: float,
          stream=None):
    """Sec. 2.6: (N, P + S + N) with N = alpha ((Phat - P) + (Shat - S)), float64 images."""
    L = _abi.lib()
    ph, n, nv, nu, sp = _image_stack(phat, "phat")
    sh, n2, nv2, nu2, ss = _image_stack(shat, "shat")
    pc = p.reshape(n, nv, nu).contiguous()
    sc = s.reshape(n, nv, nu).contiguous()
    if (n2, nv2, nu2) != (n, nv, nu) or pc.dtype != torch.float64 or sc.dtype != torch.float64:
        raise ValueError("noise: images must agree in shape and be float64")
    nz = torch.empty(n, nv, nu, dtype=torch.float64, device=ph.device)
    img = torch.empty_like(nz)
    _abi.check(L.gdrr_noise(n, nv * nu, ph.data_ptr(), sp, pc.data_ptr(), sh.data_ptr(), ss, sc.data_ptr(),
                            float(alpha), nz.data_ptr(), img.data_ptr(), _stream(stream)))
    if phat.dim() == 2:
        return nz[0], img[0]
    return nz, img


def noise_scale(n_sim: float, zeta: float, mas: float) -> float:
    """alpha = sqrt(n_sim / (zeta I)) of Sec. 2.6 (I in mAs, zeta source photons per mAs)."""
    a = C.c_double(0.0)
    _abi.check(_abi.lib().gdrr_noise_scale(float(n_sim), float(zeta), float(mas), C.byref(a)))
    return float(a.value)


def input_status(workspace: torch.Tensor, stream=None):
    """Raise GdrrError if the kernels of the last call on `workspace` met invalid
    device inputs (densities, materials, source weights); waits for the stream."""
    _abi.check(_abi.lib().gdrr_input_status(C.c_void_p(workspace.data_ptr()), _stream(stream)))


def enable_timing(on: bool = True):
    """Bracket every transport-kernel launch with HIP events on its stream."""
    _abi.check(_abi.lib().gdrr_enable_timing(1 if on else 0))


def last_kernel_ms() -> float:
    """Duration of the most recent bracketed transport kernel (waits for it)."""
    ms = C.c_float(0.0)
    _abi.check(_abi.lib().gdrr_last_kernel_ms(C.byref(ms)))
    return float(ms.value)


class JobSpec:
    """One projection of a batch: photon indices first_photon .. first_photon + n_photons - 1."""

    def __init__(self, geom, n_photons: int, job_id: int, volume: int = 0, source: int = 0,
                 first_photon: int = 0):
        self.geom, self.n_photons, self.job_id = geom, int(n_photons), int(job_id)
        self.volume, self.source, self.first_photon = int(volume), int(source), int(first_photon)


def _jobs_array(jobs: Sequence[JobSpec], planes: int = 4):
    """C job array with each job's output block of `planes` [nv][nu] images packed in order."""
    arr = (_abi.Job * len(jobs))()
    off = 0
    for k, j in enumerate(jobs):
        arr[k].volume, arr[k].source = j.volume, j.source
        arr[k].geom = geometry_struct(j.geom)
        arr[k].n_photons, arr[k].job_id, arr[k].first_photon = j.n_photons, j.job_id, j.first_photon
        arr[k].tally_offset = off
        off += planes * j.geom.nu * j.geom.nv
    return arr, off


def tuning_struct(tune) -> Optional[_abi.Tuning]:
    if tune is None:
        return None
    if isinstance(tune, _abi.Tuning):
        return tune
    return _abi.Tuning(int(tune.get("block", 0)), int(tune.get("blocks_per_cu", 0)),
                       int(tune.get("chunk", 0)), int(tune.get("defer", 0)), int(tune.get("coll_defer", 0)))


class Batch:
    """Several volumes, sources and jobs in one persistent launch."""

    def __init__(self, vols: List[DeviceVolume], phys: DevicePhysics, srcs: List[DeviceSource],
                 jobs: Sequence[JobSpec]):
        self.vols, self.phys, self.srcs, self.jobs = list(vols), phys, list(srcs), list(jobs)
        self._jobs_c, self.tally_elems = _jobs_array(self.jobs)
        self._ws = None

    def _structs(self, densities=None):
        n = len(self.vols)
        va = (_abi.Volume * n)()
        for k, v in enumerate(self.vols):
            va[k] = v.struct(None if densities is None else densities[k])
        sa = (_abi.Source * len(self.srcs))()
        for k, s in enumerate(self.srcs):
            sa[k] = s.struct()
        return va, sa, self.phys.struct()

    def workspace(self) -> torch.Tensor:
        L = _abi.lib()
        va, sa, p = self._structs()
        nbytes = int(L.gdrr_mc_project_batch_workspace(va, len(self.vols), C.byref(p), sa, len(self.srcs),
                                                      self._jobs_c, len(self.jobs)))
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.vols[0].density.device)
        return self._ws

    def set_photon_ranges(self, first_photon, n_photons):
        """Give every job the photon indices first_photon .. first_photon + n_photons - 1
        (scalars, or one value per job).  The workspace is kept, so a following
        project(resume=True) continues the fixed-point sums of the previous call."""
        k = len(self.jobs)
        firsts = list(first_photon) if hasattr(first_photon, "__len__") else [first_photon] * k
        counts = list(n_photons) if hasattr(n_photons, "__len__") else [n_photons] * k
        self.jobs = [JobSpec(j.geom, n, j.job_id, j.volume, j.source, f) for j, f, n in zip(self.jobs, firsts, counts)]
        self._jobs_c, self.tally_elems = _jobs_array(self.jobs)
        if hasattr(self, "_img_jobs"):
            del self._img_jobs
        return self

    def input_status(self, stream=None):
        """Raise GdrrError if the last transport call met invalid device inputs."""
        input_status(self.workspace(), stream)

    def tally_views(self, tallies: torch.Tensor) -> List[torch.Tensor]:
        out, off = [], 0
        for j in self.jobs:
            n = 4 * j.geom.nu * j.geom.nv
            out.append(tallies[off:off + n].view(4, j.geom.nv, j.geom.nu))
            off += n
        return out

    def primary(self, interp: bool = True, step_mm: float = 0.0, accumulate: bool = False,
                out: Optional[torch.Tensor] = None, densities=None, stream=None) -> List[torch.Tensor]:
        """Eq. 1 by ray tracing for every job: a list of [nv][nu] float64 views
        into one flat buffer (`out`, if given, holds sum(nv*nu) elements)."""
        L = _abi.lib()
        if not hasattr(self, "_img_jobs"):
            self._img_jobs = _jobs_array(self.jobs, planes=1)
        jobs_c, n = self._img_jobs
        va, sa, p = self._structs(densities)
        dev = self.vols[0].density.device
        if out is None:
            out = torch.zeros(n, dtype=torch.float64, device=dev)
        nbytes = int(L.gdrr_primary_workspace(va, len(self.vols), C.byref(p), sa, len(self.srcs), jobs_c,
                                              len(self.jobs)))
        if nbytes == 0:
            raise ValueError("invalid batch for gdrr_primary")
        if getattr(self, "_rt_ws", None) is None or self._rt_ws.numel() < nbytes:
            self._rt_ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        flags = (INTERP_DENSITY if interp else 0) | (ACCUMULATE if accumulate else 0)
        _abi.check(L.gdrr_primary(va, len(self.vols), C.byref(p), sa, len(self.srcs), jobs_c, len(self.jobs),
                                  float(step_mm), flags, out.data_ptr(), self._rt_ws.data_ptr(),
                                  self._rt_ws.numel(), _stream(stream)))
        views, off = [], 0
        for j in self.jobs:
            k = j.geom.nu * j.geom.nv
            views.append(out[off:off + k].view(j.geom.nv, j.geom.nu))
            off += k
        return views

    def majorants(self, interp: bool = True, margin: float = 2.0**-20, densities=None, stream=None):
        ms = [majorant(v, self.phys, interp, margin, None if densities is None else densities[k], stream)
              for k, v in enumerate(self.vols)]
        return torch.stack(ms)

    def project(self, seed: int = 1, interp: bool = True, sumsq: bool = True, flags: int = 0, tune=None,
                majorants: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                densities=None, resume: bool = False, stream=None) -> torch.Tensor:
        """Tallies of every job (flat float64, each job's [4][nv][nu] block in order).
        resume: continue the fixed-point sums the previous call left in the workspace
        (jobs moved on with set_photon_ranges); the output is then per source photon
        of [0, first_photon + n_photons)."""
        L = _abi.lib()
        if resume:
            flags |= RESUME
        va, sa, p = self._structs(densities)
        if out is None:
            out = torch.zeros(self.tally_elems, dtype=torch.float64, device=self.vols[0].density.device)
        ws = self.workspace()
        t = tuning_struct(tune)
        mb = None if majorants is None else majorants.contiguous().data_ptr()
        _abi.check(L.gdrr_mc_project_batch(va, len(self.vols), C.byref(p), sa, len(self.srcs), self._jobs_c,
                                           len(self.jobs), mb, seed, _flags(interp, sumsq, flags),
                                           None if t is None else C.byref(t), out.data_ptr(), ws.data_ptr(),
                                           ws.numel(), _stream(stream)))
        return out

    def backward(self, adj: torch.Tensor, majorants: torch.Tensor, volume: int = 0, seed: int = 1,
                 interp: bool = True, flags: int = 0, tune=None, grad: Optional[torch.Tensor] = None,
                 densities=None, stream=None) -> torch.Tensor:
        """adj: [n_jobs][2][nv][nu] float64 (dL/dP, dL/dS per job); returns dL/drho of `volume`."""
        L = _abi.lib()
        va, sa, p = self._structs(densities)
        v = self.vols[volume]
        if grad is None:
            grad = torch.zeros(v.shape, dtype=torch.float64, device=v.density.device)
            flags |= ACCUMULATE
        adj = adj.to(torch.float64).contiguous()
        ws = self.workspace()
        t = tuning_struct(tune)
        _abi.check(L.gdrr_mc_backward(va, len(self.vols), C.byref(p), sa, len(self.srcs), self._jobs_c,
                                      len(self.jobs), volume, majorants.contiguous().data_ptr(), seed,
                                      _flags(interp, False, flags), None if t is None else C.byref(t),
                                      adj.data_ptr(), grad.data_ptr(), ws.data_ptr(), ws.numel(),
                                      _stream(stream)))
        return grad


class GdrrProject(torch.autograd.Function):
    """(P_hat, S_hat) per job as a differentiable function of the density of
    volume 0 of a Batch.  Backward replays the forward's histories (same seed
    and majorant) and returns dL/drho from the score-function adjoint."""

    @staticmethod
    def forward(ctx, density: torch.Tensor, batch: Batch, seed: int, interp: bool, margin: float):
        densities = [density.detach().contiguous()] + [v.density for v in batch.vols[1:]]
        maj = batch.majorants(interp, margin, densities)
        tallies = batch.project(seed=seed, interp=interp, sumsq=False, majorants=maj, densities=densities)
        views = batch.tally_views(tallies)
        ps = torch.stack([torch.stack([t[0], t[2]]) for t in views])      # [n_jobs][2][nv][nu]
        ctx.batch, ctx.seed, ctx.interp = batch, seed, interp
        ctx.save_for_backward(densities[0], maj)
        return ps

    @staticmethod
    def backward(ctx, grad_ps: torch.Tensor):
        density, maj = ctx.saved_tensors
        densities = [density] + [v.density for v in ctx.batch.vols[1:]]
        g = ctx.batch.backward(grad_ps.to(torch.float64).contiguous(), maj, volume=0, seed=ctx.seed,
                               interp=ctx.interp, densities=densities)
        return g.to(density.dtype), None, None, None, None
