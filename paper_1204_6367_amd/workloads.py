"""Seeded synthetic inputs for the Monte Carlo projection step.

This module builds the *inputs* the paper's simulator consumes (Sec. 2.1 and
the Conclusion list them: a voxel phantom with a material index and a density
per voxel, mass attenuation tables per material and interaction type, a source
energy spectrum, a fluence map over the detector and a detector response
curve) together with the projection geometry.  It holds none of the transport
arithmetic: no sampling, no tracking, no scoring.  Both the GPU library and
the CPU oracle receive these arrays unchanged.

The paper's phantoms (Catphan, a head-and-neck CT), its Boone spectrum and its
measured fluence and response curves are not available, so every input here is
synthetic and seeded:

* cross sections: free-electron Klein-Nishina for Compton, K*Z_eff^4/E^3 for
  photoelectric absorption, and Rayleigh with an exponential atomic form factor
  F(x) = Z exp(-x/x0), tabulated on a 1-150 keV grid (the energy range of
  Sec. 2.4);
* spectrum: Kramers' thick-target law filtered by aluminium;
* fluence map: an isotropic point source seen by the flat detector, optionally
  multiplied by a cosine-profile aluminium bowtie (the source is defined after
  the bowtie, Sec. 2.1); optionally also the bowtie's hardening of the
  spectrum column by column (a joint source phi(E|u), one spectrum per
  detector column);
* phantoms: a water sphere in air, and ellipsoid "pelvis-like" phantoms.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

# --- physical constants ---------------------------------------------------
N_AVOGADRO = 6.02214076e23          # 1/mol
R_ELECTRON_CM = 2.8179403262e-13    # classical electron radius, cm
ME_C2_KEV = 510.99895               # electron rest energy, keV
HC_KEV_ANGSTROM = 12.398419843      # h*c in keV*Angstrom

# photoelectric constant K in mu_P/rho = K * Z_eff^4 / E^3  (cm^2/g, keV^3);
# chosen so that water's photoelectric and Compton coefficients cross near 27 keV
PHOTO_K = 1.35
# exponential form-factor scale for Rayleigh scattering, 1/Angstrom
RAYLEIGH_X0 = 0.35


@dataclasses.dataclass(frozen=True)
class Material:
    name: str
    z_over_a: float
    z_eff: float
    density: float      # nominal density, g/cm^3


MATERIALS: Dict[str, Material] = {
    "air": Material("air", 0.49919, 7.6, 0.0012),
    "water": Material("water", 0.55508, 7.4, 1.0),
    "soft_tissue": Material("soft_tissue", 0.550, 7.4, 1.03),
    "lung": Material("lung", 0.550, 7.4, 0.26),
    "bone": Material("bone", 0.530, 12.3, 1.85),
    "aluminium": Material("aluminium", 0.48181, 13.0, 2.699),
}


# --- energy grid and cross-section tables ----------------------------------
@dataclasses.dataclass
class EnergyGrid:
    e0_kev: float = 1.0
    de_kev: float = 0.5
    n_e: int = 299          # 1 .. 150 keV

    def energies(self) -> np.ndarray:
        return self.e0_kev + self.de_kev * np.arange(self.n_e, dtype=np.float64)


def klein_nishina_sigma_cm2(e_kev: np.ndarray) -> np.ndarray:
    """Total Klein-Nishina cross section per free electron, cm^2."""
    k = np.asarray(e_kev, dtype=np.float64) / ME_C2_KEV
    l2k = np.log1p(2.0 * k)
    term = ((1.0 + k) / k**2) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l2k / k) \
        + l2k / (2.0 * k) - (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2
    return 2.0 * math.pi * R_ELECTRON_CM**2 * term


def rayleigh_sigma_cm2_per_z(e_kev: np.ndarray, x0: float = RAYLEIGH_X0,
                             order: int = 96) -> np.ndarray:
    """Rayleigh cross section per atom divided by Z, with F(x) = Z exp(-x/x0).

    d(sigma)/d(Omega) = r_e^2 (1 + cos^2)/2 * F(x)^2, x = sin(theta/2)/lambda.
    Substituting cos = 1 - 2 lambda^2 x^2 gives
    sigma/Z = Z * pi r_e^2 * 4 lambda^2 * int_0^{1/lambda} (1+cos^2) e^{-2x/x0} x dx;
    the Z factor is applied by the caller.  Gauss-Legendre on [0, 1/lambda].
    """
    e = np.atleast_1d(np.asarray(e_kev, dtype=np.float64))
    t, w = np.polynomial.legendre.leggauss(order)
    out = np.empty_like(e)
    for i, ei in enumerate(e):
        lam = HC_KEV_ANGSTROM / ei
        xmax = 1.0 / lam
        # split the interval where the exponential decays: [0, min(xmax, 8 x0)] and the rest
        acc = 0.0
        edges = [0.0, min(xmax, 8.0 * x0), xmax]
        for a, b in zip(edges[:-1], edges[1:]):
            if b <= a:
                continue
            x = 0.5 * (b - a) * t + 0.5 * (b + a)
            c = 1.0 - 2.0 * lam**2 * x**2
            acc += 0.5 * (b - a) * np.sum(w * (1.0 + c * c) * np.exp(-2.0 * x / x0) * x)
        out[i] = math.pi * R_ELECTRON_CM**2 * 4.0 * lam**2 * acc
    return out


def mass_attenuation(material: Material, e_kev: np.ndarray, x0: float = RAYLEIGH_X0,
                     photo_k: float = PHOTO_K) -> np.ndarray:
    """[len(E)][3] mass attenuation (cm^2/g): Rayleigh, Compton, photoelectric."""
    e = np.asarray(e_kev, dtype=np.float64)
    ne = N_AVOGADRO * material.z_over_a           # electrons per gram
    mu_c = ne * klein_nishina_sigma_cm2(e)
    mu_r = ne * material.z_eff * rayleigh_sigma_cm2_per_z(e, x0)
    mu_p = photo_k * material.z_eff**4 / e**3
    return np.stack([mu_r, mu_c, mu_p], axis=-1)


def cross_section_table(names: Sequence[str], grid: EnergyGrid = EnergyGrid(),
                        x0: float = RAYLEIGH_X0) -> np.ndarray:
    """float32 [n_mat][n_e][3] table (Rayleigh, Compton, photoelectric), cm^2/g."""
    e = grid.energies()
    tab = np.stack([mass_attenuation(MATERIALS[n], e, x0) for n in names])
    return tab.astype(np.float32)


# --- source ----------------------------------------------------------------
def kramers_spectrum(kvp: float = 120.0, al_mm: float = 2.5, bin_kev: float = 1.0,
                     e_min_kev: float = 1.0):
    """Kramers photon-number spectrum (kvp - E)/E filtered by aluminium.

    Returns (energies at bin centres, float32 probabilities summing to 1)."""
    edges = np.arange(e_min_kev, kvp + 1e-9, bin_kev)
    e = 0.5 * (edges[:-1] + edges[1:])
    al = MATERIALS["aluminium"]
    mu_al = mass_attenuation(al, e).sum(axis=-1) * al.density      # 1/cm
    phi = (kvp - e) / e * np.exp(-mu_al * al_mm * 0.1)
    phi = np.clip(phi, 0.0, None)
    phi /= phi.sum()
    return e.astype(np.float32), phi.astype(np.float32)


def mono_spectrum(e_kev: float = 60.0):
    return np.array([e_kev], np.float32), np.array([1.0], np.float32)


@dataclasses.dataclass
class Geometry:
    """Cone-beam geometry of Sec. 2.1 (lengths in mm, angles in radians)."""
    sad_mm: float = 1000.0
    aid_mm: float = 500.0          # axis-to-imager distance; SDD = SAD + AID for theta = 0
    phi_rad: float = 0.0
    theta_rad: float = 0.0
    nu: int = 64
    nv: int = 48
    du_mm: float = 4.0
    dv_mm: float = 4.0

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def fluence_map(geom: Geometry, bowtie_mm: float = 0.0, spectrum=None,
                quad: int = 4) -> np.ndarray:
    """Per-pixel probabilities [nv][nu] (float32, sum 1) of the aim point.

    Geometric factor: an isotropic point source at distance SDD from the flat
    detector sends d(Omega) = SDD / (SDD^2 + u^2 + v^2)^{3/2} du dv per area.
    Bowtie (optional): aluminium thickness t = bowtie_mm (1 - cos(pi g/(2 gmax)))
    at fan angle g toward u; transmission averaged over `spectrum`."""
    sdd = geom.sad_mm + geom.aid_mm
    t, w = np.polynomial.legendre.leggauss(quad)
    w = w / 2.0
    ue = (np.arange(geom.nu) - geom.nu / 2.0) * geom.du_mm
    ve = (np.arange(geom.nv) - geom.nv / 2.0) * geom.dv_mm
    uq = (ue[:, None] + (0.5 * (t + 1.0))[None, :] * geom.du_mm)     # [nu][q]
    vq = (ve[:, None] + (0.5 * (t + 1.0))[None, :] * geom.dv_mm)     # [nv][q]
    U = uq[None, :, None, :]
    V = vq[:, None, :, None]
    geo = sdd / (sdd**2 + U**2 + V**2) ** 1.5                         # [nv][nu][q][q]
    if bowtie_mm > 0.0:
        if spectrum is None:
            raise ValueError("bowtie needs the spectrum it hardens")
        trans = (np.asarray(spectrum[1], np.float64)[None, None, :] *
                 _bowtie_transmission(geom, bowtie_mm, spectrum[0], uq)).sum(-1)  # [nu][q]
        geo = geo * trans[None, :, None, :]
    f = (geo * w[None, None, :, None] * w[None, None, None, :]).sum(axis=(2, 3))
    f = f * geom.du_mm * geom.dv_mm
    f /= f.sum()
    return f.astype(np.float32)


def _bowtie_transmission(geom: Geometry, bowtie_mm: float, spec_e, uq: np.ndarray) -> np.ndarray:
    """exp(-mu_Al(E) t(u)) at detector abscissae uq (any shape) for every
    channel energy: [*uq.shape, n_spec].  t = bowtie_mm (1 - cos(pi g / (2 gmax)))
    at fan angle g toward u; gmax is the fan angle of the detector edge."""
    sdd = geom.sad_mm + geom.aid_mm
    al = MATERIALS["aluminium"]
    mu_al = mass_attenuation(al, np.asarray(spec_e, np.float64)).sum(-1) * al.density * 0.1  # 1/mm
    gmax = math.atan(0.5 * geom.nu * geom.du_mm / sdd)
    gam = np.arctan(np.abs(uq) / sdd)
    thick = bowtie_mm * (1.0 - np.cos(0.5 * math.pi * gam / gmax))
    return np.exp(-mu_al * thick[..., None])


def bowtie_spectra(geom: Geometry, bowtie_mm: float, spectrum, quad: int = 4) -> np.ndarray:
    """Joint source after a bowtie: the spectrum of the photons aimed at each
    detector column, [nu][n_spec] float32, each row summing to 1.

    Row iu is phi(E) times the bowtie transmission at E averaged over the
    column (Gauss-Legendre in u, weighted by the point source's solid angle
    integrated over v); the marginal of the aim pixel is `fluence_map` with
    the same bowtie."""
    sdd = geom.sad_mm + geom.aid_mm
    t, w = np.polynomial.legendre.leggauss(quad)
    w = w / 2.0
    ue = (np.arange(geom.nu) - geom.nu / 2.0) * geom.du_mm
    ve = (np.arange(geom.nv) - geom.nv / 2.0) * geom.dv_mm
    uq = ue[:, None] + (0.5 * (t + 1.0))[None, :] * geom.du_mm          # [nu][q]
    vq = (ve[:, None] + (0.5 * (t + 1.0))[None, :] * geom.dv_mm).ravel()
    col = (sdd / (sdd**2 + uq[..., None]**2 + vq**2) ** 1.5) @ np.tile(w, geom.nv)   # [nu][q]
    trans = _bowtie_transmission(geom, bowtie_mm, spectrum[0], uq)       # [nu][q][n_spec]
    rows = np.asarray(spectrum[1], np.float64) * ((col * w)[..., None] * trans).sum(1)
    rows /= rows.sum(1, keepdims=True)
    return rows.astype(np.float32)


# --- phantoms ----------------------------------------------------------------
@dataclasses.dataclass
class Phantom:
    density: np.ndarray        # float32 [nz][ny][nx], g/cm^3
    material: np.ndarray       # uint8   [nz][ny][nx]
    spacing_mm: tuple          # (dx, dy, dz)
    materials: List[str]       # names, indexed by the material byte

    @property
    def shape(self):
        return self.density.shape


def _centres(n: int, d: float) -> np.ndarray:
    return ((np.arange(n) + 0.5) - n / 2.0) * d


def sphere_phantom(n: int = 64, d_mm: float = 2.0, radius_mm: float = 50.0,
                   inner: str = "water", outer: str = "air") -> Phantom:
    """Cube of n^3 voxels centred on the isocentre; voxels whose centre lies
    within `radius_mm` of the centre take the inner material."""
    c = _centres(n, d_mm)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = x * x + y * y + z * z <= radius_mm**2
    names = [outer, inner]
    mat = inside.astype(np.uint8)
    dens = np.where(inside, MATERIALS[inner].density, MATERIALS[outer].density).astype(np.float32)
    return Phantom(dens, mat, (d_mm, d_mm, d_mm), names)


def box_phantom(shape, spacing_mm, material: str = "water",
                density: Optional[float] = None) -> Phantom:
    nz, ny, nx = shape
    rho = MATERIALS[material].density if density is None else density
    return Phantom(np.full(shape, rho, np.float32), np.zeros(shape, np.uint8),
                   tuple(spacing_mm), [material])


ELLIPSOID_MATERIALS = ["air", "soft_tissue", "bone", "lung"]


def ellipsoid_phantom(shape, spacing_mm, seed: int, n_inner: int = 11) -> Phantom:
    """Pelvis-like phantom: a soft-tissue body ellipsoid with semi-axes
    (0.42 X, 0.30 Y, 0.45 Z) of the volume's extents, then `n_inner` ellipsoids
    (centres uniform inside 0.7 x the body, semi-axes U(10, 60) mm, uniformly
    random orientation, material bone/lung/soft tissue with probabilities
    0.45/0.20/0.35) painted in order over air.  numpy PCG64 with `seed`."""
    nz, ny, nx = shape
    dx, dy, dz = spacing_mm
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = np.array([nx * dx, ny * dy, nz * dz])
    body = np.array([0.42, 0.30, 0.45]) * ext
    ell = [(np.zeros(3), body, np.eye(3), 1)]
    choices = np.array([2, 3, 1])
    probs = np.array([0.45, 0.20, 0.35])
    for _ in range(n_inner):
        while True:
            p = rng.uniform(-1.0, 1.0, 3)
            if p @ p <= 1.0:
                break
        centre = 0.7 * body * p
        axes = rng.uniform(10.0, 60.0, 3)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        mat = int(rng.choice(choices, p=probs))
        ell.append((centre, axes, q, mat))
    material = np.zeros(shape, np.uint8)
    xc, yc, zc = _centres(nx, dx), _centres(ny, dy), _centres(nz, dz)
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    for k in range(nz):
        sl = material[k]
        for centre, axes, rot, mat in ell:
            if abs(zc[k] - centre[2]) > axes.max():
                continue
            rel = np.stack([X - centre[0], Y - centre[1], np.full_like(X, zc[k] - centre[2])], -1)
            loc = rel @ rot                      # coordinates in the ellipsoid frame
            inside = ((loc / axes) ** 2).sum(-1) <= 1.0
            sl[inside] = mat
    dens_by_mat = np.array([MATERIALS[n].density for n in ELLIPSOID_MATERIALS], np.float32)
    density = dens_by_mat[material]
    return Phantom(density, material, tuple(spacing_mm), list(ELLIPSOID_MATERIALS))


def perturb_density(ph: Phantom, seed: int, amplitude: float = 0.05) -> Phantom:
    """rho* = rho (1 + amplitude U(-1, 1)) per voxel, materials unchanged."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(-1.0, 1.0, ph.density.shape)
    dens = (ph.density.astype(np.float64) * (1.0 + amplitude * f)).astype(np.float32)
    return Phantom(dens, ph.material.copy(), ph.spacing_mm, list(ph.materials))


# --- physics bundle ---------------------------------------------------------
@dataclasses.dataclass
class Physics:
    mu_mass: np.ndarray                 # float32 [n_mat][n_e][3]
    grid: EnergyGrid
    response: Optional[np.ndarray] = None   # float32 [n_e] keV, None => r(E) = E
    rayleigh_x0: float = RAYLEIGH_X0
    e_cut_kev: float = 1.0


def physics_for(ph: Phantom, grid: EnergyGrid = EnergyGrid(), response=None) -> Physics:
    return Physics(cross_section_table(ph.materials, grid), grid, response)


@dataclasses.dataclass
class Source:
    spec_e: np.ndarray      # float32 [n_spec], keV
    spec_p: np.ndarray      # float32 [n_spec], or [nu][n_spec]: one spectrum per detector column
    fluence: np.ndarray     # float32 [nv][nu]


@dataclasses.dataclass
class Problem:
    phantom: Phantom
    physics: Physics
    source: Source
    geom: Geometry
    n_photons: int
    seed: int = 1
    job_id: int = 0
    interp: bool = True


# --- the workloads ----------------------------------------------------------
PELVIS_DET = dict(nu=256, nv=192, du_mm=1.552, dv_mm=1.552)


def sphere_problem(n_photons: int = 1_000_000) -> Problem:
    """64^3 at 2 mm, water sphere r = 50 mm in air, 60 keV, 64x48 detector of 4 mm."""
    ph = sphere_phantom()
    geom = Geometry(nu=64, nv=48, du_mm=4.0, dv_mm=4.0)
    e, p = mono_spectrum(60.0)
    src = Source(e, p, fluence_map(geom))
    return Problem(ph, physics_for(ph), src, geom, n_photons, seed=1)


def pelvis_source(geom: Geometry, joint: bool = False):
    """120 kVp + 2.5 mm Al behind a 30 mm Al bowtie.  joint=False: one
    spectrum for every direction (the bowtie only shapes the fluence map);
    joint=True: one hardened spectrum per detector column."""
    spec = kramers_spectrum(120.0, 2.5, 1.0)
    rows = bowtie_spectra(geom, 30.0, spec) if joint else spec[1]
    return Source(spec[0], rows, fluence_map(geom, bowtie_mm=30.0, spectrum=spec))


def pelvis_problem(n_photons: int = 100_000_000, shape=(160, 256, 256),
                   spacing=(1.95, 1.95, 2.5), seed_phantom: int = 11) -> Problem:
    """256x256x160 ellipsoid phantom, 120 kVp + 2.5 mm Al, 30 mm Al bowtie,
    256x192 detector of 1.552 mm."""
    ph = ellipsoid_phantom(shape, spacing, seed_phantom)
    geom = Geometry(**PELVIS_DET)
    return Problem(ph, physics_for(ph), pelvis_source(geom), geom, n_photons, seed=1)


def adjoint_problem(n_photons: int = 10_000_000):
    """128x128x96 at 3 mm (ellipsoid generator, seed 31); target densities
    perturbed by +-5 % (seed 32)."""
    ph = ellipsoid_phantom((96, 128, 128), (3.0, 3.0, 3.0), 31)
    target = perturb_density(ph, 32)
    geom = Geometry(**PELVIS_DET)
    prob = Problem(ph, physics_for(ph), pelvis_source(geom), geom, n_photons, seed=1)
    return prob, target


MULTI_PHANTOMS = [
    # (shape [nz,ny,nx], spacing (dx,dy,dz), seed, n_angles, photons per angle)
    ((256, 512, 512), (0.98, 0.98, 0.98), 41, 60, 100_000_000),
    ((160, 256, 256), (1.95, 1.95, 1.95), 42, 120, 30_000_000),
    ((64, 128, 128), (4.0, 4.0, 4.0), 43, 360, 10_000_000),
]


def angles(n: int) -> np.ndarray:
    """n gantry angles evenly spaced over a full turn, radians."""
    return 2.0 * math.pi * np.arange(n) / n
