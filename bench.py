"""Benchmark of the gfx950 Monte Carlo projection step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4]

One step runs every stage of the hot path over one batch of synthetic input:
majorants, source tables, the persistent batched transport kernel with its
scoring and finalisation, and (for workloads with a loss) the path-replay
adjoint.  Inputs are resident in HBM before the timed region.  Prints ONE
JSON line with the whole-step histories/s, the roofline of the transport
kernel (timed with HIP events on its own stream, inside the library) and the
CPU oracle timed on a bounded sample of the same workload.  Beside the step,
outside its timing, the ray-tracing primary (Eq. 1) of the same jobs, the
denoising of the step's scatter tallies (Eq. 5) and the noise assembly
(Sec. 2.6) are timed and reported under "raytrace" and "denoise" with their
own rooflines and oracle rates.

Workloads (synthetic, seeded; sizes of the paper's CBCT setting):
  c1  one projection: 256x256x160 ellipsoid phantom, 120 kVp + bowtie, 1e8 photons
  c2  360 angles of the c1 phantom, 1e7 photons each, one persistent launch
  c3  adjoint: 128x128x96 phantom, 1e7 photons, loss 0.5 ||S - S*||^2
  c4  three phantoms (512^2x256, 256^2x160, 128^2x64) at 60/120/360 angles,
      1e8/3e7/1e7 photons per angle, then the adjoint of the second phantom
      at 30 of its angles
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon histories/sec (fwd, batched angles) + adjoint histories/sec, 1×MI355X"

# MI355X peaks used for the roofline fractions
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # 32-bit VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz

# Work model of one history (algorithmic units; see the design notes), in
# slots of a full-rate 32-bit integer VALU lane operation (the 39.3 T/s peak).
# Costs of the instruction classes as measured on gfx950 by
# paper_1204_6367_amd/calib/issue_rate (relative to a chain of float32 FMAs):
# integer operations, 32x32-bit products (v_mul_hi_u32, v_mad_u64_u32)
# included, 1 slot; float32 add, mul, fma, min, compare with vector operands
# 0.6 (they issue at about twice the integer rate; 1.05 when an operand is a
# scalar register); transcendentals (log, exp, rcp, rsq, sqrt, sin, cos) 2.3.
SLOTS_INT = 1.0
SLOTS_F32 = 0.6
SLOTS_TRANS = 2.3


def slots(i=0, f=0, t=0):
    """Slots of i integer, f float32 and t transcendental operations."""
    return i * SLOTS_INT + f * SLOTS_F32 + t * SLOTS_TRANS


SLOTS_PHILOX = slots(i=10 * (2 + 2))                  # per round: two 32x32->64 products, two 3-way xors
# free flights come in pairs sharing one Philox block (counted per history below)
SLOTS_FLIGHT_IN = slots(i=10, f=31, t=1)              # uniforms, -ln u, move, cell-record trilinear, lookup+ladder
SLOTS_FLIGHT_OUT = slots(i=7, f=27, t=2)              # the escaping flight: -ln u, detector intersection
SLOTS_TRY = SLOTS_PHILOX + slots(i=8, f=25, t=3)      # one angular-sampler try (KN: sqrt or none, two rcp)
SLOTS_SELECT = slots(i=2, f=4)                        # interaction type, at every real collision
SLOTS_COLLISION = SLOTS_SELECT + slots(i=11, f=54, t=10)   # + sampler constants, rotation, energy cache
SLOTS_BOX_EXIT = slots(i=6, f=28, t=3)                # single majorant only: distance to the box
SLOTS_SOURCE = 2 * SLOTS_PHILOX + slots(i=50, f=55, t=4)   # two blocks, CDFs (fp64), aim point, box entry
# local majorants: every pair of flights first sets up its walk (cube coordinates,
# three reciprocals, steps, exit-face distances; the second flight goes on along
# the same walk), then each flight visits cubes (the one it starts in, and
# one per face crossed): record word address and load, the bound from the row of
# the material-set table it names, spend or stop, advance, step the cube index
SLOTS_WALK = slots(i=30, f=42, t=3)
SLOTS_CUBE = slots(i=20, f=23)
BYTES_CUBE = 4
BYTES_FLIGHT_IN = 8 * 4 + 1                            # eight density corners + the containing voxel's material
BYTES_SOURCE = 2 * (2 * 8 + 4) + 4                     # CDF + guide reads for energy and pixel, energy
BYTES_SCORE = 8                                        # one fixed-point atomic


def work_per_history(stats, n):
    """Average algorithmic VALU slots and bytes per history from oracle counts."""
    h = float(n)
    entered = h * 1.0
    flights = stats["steps"] / h
    real = stats["real"] / h
    tries = stats["tries"] / h
    scatter_events = (stats["compton"] + stats["rayleigh"]) / h
    scored = (stats["classes"]["primary"] + stats["classes"]["scatter"]) / h
    # every history that entered the phantom ends its last flight by escaping
    # (or is absorbed/cut at a collision); in-box flights = flights - escapes
    escapes = (stats["classes"]["primary"] + stats["classes"]["scatter"] + stats["classes"]["missed"]) / h
    inbox = max(flights - escapes, 0.0)
    pairs = 0.5 * (flights + real)                     # a real collision ends a pair early
    crossings = stats.get("crossings", 0.0) / h
    cubes = (crossings + flights) if crossings > 0 else 0.0
    local = crossings > 0
    slots = (pairs * SLOTS_PHILOX + inbox * SLOTS_FLIGHT_IN + escapes * SLOTS_FLIGHT_OUT + tries * SLOTS_TRY
             + real * SLOTS_SELECT + scatter_events * (SLOTS_COLLISION - SLOTS_SELECT + (0 if local else SLOTS_BOX_EXIT))
             + SLOTS_SOURCE + (pairs * SLOTS_WALK + cubes * SLOTS_CUBE if local else 0.0))
    nbytes = inbox * BYTES_FLIGHT_IN + BYTES_SOURCE + scored * BYTES_SCORE + cubes * BYTES_CUBE
    return dict(slots=slots, bytes=nbytes, flights=flights, inbox_flights=inbox, real=real, tries=tries,
                cube_visits=cubes)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha() -> str:
    """Hash of the HIP sources: measured traffic is valid only for this kernel."""
    import hashlib
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1204_6367_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


TRAFFIC_PATH = None
GATHER_PATH = os.path.join(ROOT, "profiles", "gather_rates_gfx950.json")
GATHER_RECORD = 32                 # bytes of one cell record: the gather of a free flight inside a phantom


def gather_peak(rates, ws_bytes):
    """Measured random-gather rate (GB/s) of records of one size for a
    working set: the rate at the smallest measured working set that holds it
    (the largest measured one beyond)."""
    pts = sorted(rates)
    for ws, gbs in pts:
        if ws >= ws_bytes:
            return gbs
    return pts[-1][1]


def gather_roofline(path, batch, inbox_flights, histories_per_s):
    """The transport's cell-record gathers against the random-gather rate
    measured at each phantom's working set (its cell records), the rates
    combined harmonically with the photons each phantom gets; None without
    the measurement."""
    try:
        rates = json.load(open(path))["rates"][str(GATHER_RECORD)]
    except (OSError, ValueError, KeyError):
        return None
    photons = {}
    for j in batch.jobs:
        photons[j.volume] = photons.get(j.volume, 0) + j.n_photons
    total = float(sum(photons.values()))
    inv, sets = 0.0, []
    for v, n in sorted(photons.items()):
        nz, ny, nx = batch.vols[v].density.shape
        ws = (nx + 1) * (ny + 1) * (nz + 1) * GATHER_RECORD
        sets.append(round(ws / 1e9, 3))
        inv += n / total / gather_peak(rates, ws)
    peak = 1.0 / inv
    ach = inbox_flights * GATHER_RECORD * histories_per_s / 1e9
    return dict(bound="gather", achieved=round(ach, 1), peak=round(peak, 1), unit="GB/s", frac=round(ach / peak, 4),
                record_bytes=GATHER_RECORD, working_sets_gb=sets)


def measured_traffic(path, workload, kernel=None):
    """Memory-side bytes per launch of a kernel from rocprofv3 FETCH_SIZE +
    WRITE_SIZE (scaled by the copy calibration), if they were taken on the
    current kernel sources.  `kernel` selects a secondary record
    ("raytrace", "denoise") of the workload."""
    if not path or not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_sources_sha():
        return None
    if kernel is not None:
        rec = rec.get("others", {}).get(kernel)
        if not rec:
            return None
    return round(rec["fetch_bytes"] + rec["write_bytes"], 0)


def measured_counters(path, workload, kernel=None):
    """rocprofv3 counter readings of a kernel (active-lane fraction, VALU
    instruction rate and the issue-utilisation bounds priced from the
    issue-rate calibration, L2 hit rate), if taken on the current kernel
    sources; `kernel` selects a secondary record ("adjoint", ...)."""
    if not path or not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_sha") != kernel_sources_sha():
        return None
    if kernel is not None:
        rec = rec.get("others", {}).get(kernel)
    if not rec or "counters" not in rec:
        return None
    c = {k: v for k, v in rec["counters"].items() if k != "duration_ms"}
    c["kernel"] = rec["kernel"]
    return c


TUNE_MODE = "auto"
TUNE_CACHE = None
MAJORANT = "local"
CUBE_MM = 40.0
SOURCE = "factorised"        # or "joint": one spectrum per detector column


ADJ_MARGIN = 0.1            # the adjoint volume's majorant margin (null-collision terms stay bounded)
ADJ_RHO_MIN = 0.05          # and its cubes' density floor, g/cm^3 (float32 collision points in air cubes)


def apply_majorant(vol, margin, rho_min=0.0):
    """Local majorants on cubes of about CUBE_MM (or the single per-energy majorant)."""
    if MAJORANT == "local":
        vol.local_majorants(max(1, int(round(CUBE_MM / min(vol.spacing_mm)))), margin, rho_min)


def majorant_desc(vols):
    if MAJORANT != "local":
        return "global"
    return f"local, cubes of {[v.macro for v in vols]} voxels (~{CUBE_MM:g} mm)"


def autotune_for(batch, mode="forward", volume=0):
    """Launch shape from the autotuner's cache for this workload class, or (not
    cached) from a fresh search on 2 % of the photons; untimed setup either way."""
    from paper_1204_6367_amd import autotune
    if TUNE_MODE == "default":
        return None
    t = time.time()
    best = autotune.autotune(batch, fraction=0.02, min_photons=200_000, cache=TUNE_CACHE,
                             force=TUNE_MODE == "search", mode=mode, volume=volume)
    log(f"autotune ({mode}) {best} in {time.time() - t:.1f}s")
    return best


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
SPECTRUM_DESC = {"factorised": "120 kVp Kramers + 2.5 mm Al, bowtie 30 mm Al",
                 "joint": "120 kVp Kramers + 2.5 mm Al, bowtie 30 mm Al hardening each detector column's spectrum"}


def build_workload(name, api, W, torch):
    """Returns dict(step=callable, fwd_histories, adj_histories, oracle_sample=callable, info)."""
    if name in ("c1", "c2"):
        prob = W.pelvis_problem(100_000_000)
        if SOURCE == "joint":
            prob.source = W.pelvis_source(prob.geom, joint=True)
        vol, phys, src = api.upload(prob)
        apply_majorant(vol, 2.0**-20)
        if name == "c1":
            jobs = [api.JobSpec(prob.geom, 100_000_000, 0)]
        else:
            jobs = [api.JobSpec(prob.geom.replace(phi_rad=float(a)), 10_000_000, k)
                    for k, a in enumerate(np.deg2rad(np.arange(360.0)))]
        batch = api.Batch([vol], phys, [src], jobs)
        tallies = torch.zeros(batch.tally_elems, dtype=torch.float64, device="cuda")
        fwd = sum(j.n_photons for j in jobs)
        tune = autotune_for(batch)

        def step():
            maj = batch.majorants(True)
            batch.project(seed=1, majorants=maj, out=tallies, tune=tune)
            return [api.last_kernel_ms()]

        samples = [(prob, float(jobs[k].geom.phi_rad), jobs[k].job_id, vol.macro, vol.macro_margin,
                    vol.macro_rho_min) for k in (0, len(jobs) // 2)]
        return dict(step=step, fwd=fwd, adj=0, samples=samples, adjoint=None, batch=batch, prob_of=lambda k: prob,
                    tallies=tallies,
                    config=dict(workload=name, phantom="256x256x160 @1.95x1.95x2.5mm ellipsoids",
                                angles=len(jobs), photons_per_angle=jobs[0].n_photons,
                                detector="256x192 @1.552mm", spectrum=SPECTRUM_DESC[SOURCE],
                                tuning=tune, majorant=majorant_desc([vol])))
    if name in ("c3", "c4"):
        if name == "c3":
            prob, target = W.adjoint_problem(10_000_000)
            phantoms = [(prob.phantom, target)]
            plan = [(0, 1, 10_000_000)]                      # (volume, n_angles, photons)
            adj_vol, adj_jobs_every = 0, 1
        else:
            phantoms = []
            plan = []
            for v, (shape, sp, seed, n_ang, nph) in enumerate(W.MULTI_PHANTOMS):
                t = time.time()
                ph = W.ellipsoid_phantom(shape, sp, seed)
                log(f"phantom {v} {shape} built in {time.time() - t:.1f}s")
                phantoms.append((ph, W.perturb_density(ph, seed + 100) if v == 1 else None))
                plan.append((v, n_ang, nph))
            adj_vol, adj_jobs_every = 1, 4
        geom = W.Geometry(**W.PELVIS_DET)
        srcw = W.pelvis_source(geom, joint=SOURCE == "joint")
        physw = W.physics_for(phantoms[0][0])
        vols = [api.DeviceVolume(ph.density, ph.material, ph.spacing_mm) for ph, _ in phantoms]
        dphys = api.DevicePhysics(physw.mu_mass, physw.grid.e0_kev, physw.grid.de_kev)
        dsrc = api.DeviceSource(srcw.spec_e, srcw.spec_p, srcw.fluence)
        jobs, adj_idx = [], []
        jid = 0
        for v, n_ang, nph in plan:
            for a in range(n_ang):
                phi = 2.0 * math.pi * a / n_ang
                if v == adj_vol and a % adj_jobs_every == 0:
                    adj_idx.append(len(jobs))
                jobs.append(api.JobSpec(geom.replace(phi_rad=phi), nph, jid, volume=v))
                jid += 1
        batch = api.Batch(vols, dphys, [dsrc], jobs)
        adj_batch = api.Batch(vols, dphys, [dsrc], [jobs[k] for k in adj_idx])
        margins = [ADJ_MARGIN if v == adj_vol else 2.0**-20 for v in range(len(vols))]
        for k, v in enumerate(vols):
            apply_majorant(v, margins[k], ADJ_RHO_MIN if k == adj_vol else 0.0)
        # target tallies S* of the perturbed phantom (Philox seed 2), not timed
        tgt_vol = api.DeviceVolume(phantoms[adj_vol][1].density, phantoms[adj_vol][1].material,
                                   phantoms[adj_vol][1].spacing_mm)
        tvols = list(vols)
        tvols[adj_vol] = tgt_vol
        tb = api.Batch(tvols, dphys, [dsrc], [jobs[k] for k in adj_idx])
        t_tally = tb.project(seed=2, sumsq=False)
        s_target = torch.stack([t[2] for t in tb.tally_views(t_tally)])
        tallies = torch.zeros(batch.tally_elems, dtype=torch.float64, device="cuda")
        grad = torch.zeros(vols[adj_vol].shape, dtype=torch.float64, device="cuda")
        fwd = sum(j.n_photons for j in jobs)
        adjh = sum(jobs[k].n_photons for k in adj_idx)
        state = {}
        tune = autotune_for(batch)
        adj_tune = autotune_for(adj_batch, mode="backward", volume=adj_vol)

        def step():
            maj = torch.stack([api.majorant(v, dphys, True, margins[k]) for k, v in enumerate(vols)])
            batch.project(seed=1, sumsq=False, majorants=maj, out=tallies, tune=tune)
            ms_f = api.last_kernel_ms()
            views = batch.tally_views(tallies)
            s_now = torch.stack([views[k][2] for k in adj_idx])
            adj = torch.zeros(len(adj_idx), 2, geom.nv, geom.nu, dtype=torch.float64, device="cuda")
            adj[:, 1] = s_now - s_target                       # d(0.5||S - S*||^2)/dS
            adj_batch.backward(adj, maj, volume=adj_vol, seed=1, grad=grad, tune=adj_tune)
            ms_b = api.last_kernel_ms()
            state["loss"] = 0.5 * float(((s_now - s_target) ** 2).sum())
            return [ms_f, ms_b]

        samples = []
        for v, n_ang, nph in plan:
            k = next(i for i, j in enumerate(jobs) if j.volume == v)
            ph = phantoms[v][0]
            samples.append((W.Problem(ph, physw, srcw, jobs[k].geom, nph), float(jobs[k].geom.phi_rad),
                            jobs[k].job_id, vols[v].macro, vols[v].macro_margin, vols[v].macro_rho_min))
        adjoint = dict(problem=W.Problem(phantoms[adj_vol][0], physw, srcw, jobs[adj_idx[0]].geom, 1),
                       job_id=jobs[adj_idx[0]].job_id, margin=ADJ_MARGIN, macro=vols[adj_vol].macro,
                       rho_min=vols[adj_vol].macro_rho_min)
        cfg = dict(workload=name, angles=len(jobs), adjoint_angles=len(adj_idx), tuning=tune, adjoint_tuning=adj_tune,
                   majorant=majorant_desc(vols),
                   detector="256x192 @1.552mm", spectrum=SPECTRUM_DESC[SOURCE],
                   phantoms=[f"{'x'.join(map(str, ph.shape[::-1]))} @{ph.spacing_mm[0]}mm" for ph, _ in phantoms],
                   photons_per_angle=[p[2] for p in plan])
        def prob_of(k):
            return W.Problem(phantoms[jobs[k].volume][0], physw, srcw, jobs[k].geom, 0)

        return dict(step=step, fwd=fwd, adj=adjh, samples=samples, adjoint=adjoint, config=cfg, batch=batch,
                    prob_of=prob_of, tallies=tallies)
    raise SystemExit(f"unknown workload {name}")


# ---------------------------------------------------------------------------
# Ray-tracing primary (Eq. 1) over the same jobs: measured beside the step
# ---------------------------------------------------------------------------
# per interval: bounds and midpoint (5), lattice coordinates (3 FMA),
# floor/convert/clamp (12), fractions (6), cell address (4), trilinear (14),
# accumulate (2), loop (2)
SLOTS_RT_INTERVAL = slots(i=13, f=33)
# Compulsory memory traffic per image: the volume's density and material
# (5 bytes per voxel, read once; an upper bound, as the cone may miss part of
# the volume) and the float64 image.  Rays of one tile and successive intervals
# of one ray share voxels, so bytes gathered per interval (40) are mostly cache hits.
BYTES_RT_VOXEL = 5
BYTES_RT_PIXEL = 8


def rt_intervals(batch, dl_of):
    """Intervals the ray tracer evaluates (ray parts inside the phantom box,
    cut at multiples of dl from the source), counted on the host in float64."""
    total = 0
    for j in batch.jobs:
        g, v = j.geom, batch.vols[j.volume]
        nz, ny, nx = v.shape
        half = 0.5 * np.array([nx, ny, nz]) * np.array(v.spacing_mm)
        cq, sq = math.cos(g.phi_rad + g.theta_rad), math.sin(g.phi_rad + g.theta_rad)
        S = -g.sad_mm * np.array([math.cos(g.phi_rad), math.sin(g.phi_rad), 0.0])
        P = g.aid_mm * np.array([cq, sq, 0.0])
        eu = np.array([-sq, cq, 0.0])
        uc = (np.arange(g.nu) + 0.5 - 0.5 * g.nu) * g.du_mm
        vc = (np.arange(g.nv) + 0.5 - 0.5 * g.nv) * g.dv_mm
        D = P[None, None] + uc[None, :, None] * eu[None, None] + vc[:, None, None] * np.array([0, 0, 1.0])[None, None]
        d = (D - S).reshape(-1, 3)
        ln = np.linalg.norm(d, axis=1)
        d /= ln[:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (-half[None] - S[None]) / d
            tb = (half[None] - S[None]) / d
        t0 = np.maximum(np.nanmax(np.minimum(ta, tb), axis=1), 0.0)
        t1 = np.minimum(np.nanmin(np.maximum(ta, tb), axis=1), ln)
        dl = dl_of(v)
        hit = t1 > t0
        total += int((np.ceil(t1[hit] / dl) - np.floor(t0[hit] / dl)).sum())
    return total


def raytrace_leg(wl, api, torch, steps, cpu):
    batch = wl["batch"]
    dl_of = lambda v: 0.5 * min(v.spacing_mm)
    batch.primary()                                   # workspace and cell records
    torch.cuda.synchronize()
    ms, walls = [], []
    for _ in range(max(steps, 1)):
        t = time.perf_counter()
        batch.primary()
        ms.append(api.last_kernel_ms())
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t) * 1e3)
    kms = float(np.mean(ms))
    rays = sum(j.geom.nu * j.geom.nv for j in batch.jobs)
    iv = rt_intervals(batch, dl_of)
    alu = iv * SLOTS_RT_INTERVAL / (kms * 1e-3) / 1e12
    nbytes = sum(BYTES_RT_VOXEL * int(np.prod(batch.vols[j.volume].shape)) + BYTES_RT_PIXEL * j.geom.nu * j.geom.nv
                 for j in batch.jobs)
    gbs = nbytes / (kms * 1e-3) / 1e9
    tr = measured_traffic(TRAFFIC_PATH, wl["config"]["workload"], "raytrace")
    ra = dict(bound="alu", achieved=round(alu, 3), peak=round(ALU_PEAK_TOPS, 2), unit="Tops/s",
              frac=round(alu / ALU_PEAK_TOPS, 4), traffic=tr)
    rh = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
              frac=round(gbs / HBM_PEAK_GBS, 4), traffic=tr)
    out = dict(images=len(batch.jobs), kernel_ms=round(kms, 3), wall_ms=round(float(np.mean(walls)), 3),
               images_per_s=round(len(batch.jobs) / (kms * 1e-3), 1), rays_per_s=round(rays / (kms * 1e-3), 1),
               intervals=iv, intervals_per_s=round(iv / (kms * 1e-3), 1), compulsory_bytes=nbytes,
               roofline=ra if ra["frac"] >= rh["frac"] else rh, roofline_other=rh if ra["frac"] >= rh["frac"] else ra)
    if cpu:
        import oracle
        k = 0
        p = oracle.Problem.from_workload(wl["prob_of"](k), phi_rad=batch.jobs[k].geom.phi_rad)
        rng = np.random.default_rng(0)
        g = batch.jobs[k].geom
        n = 256
        while True:
            pix = rng.choice(g.nu * g.nv, min(n, g.nu * g.nv), replace=False)
            t = time.time()
            oracle.primary_raytrace(p, pixels=pix)
            dt = time.time() - t
            if dt > 2.0 or n >= g.nu * g.nv:
                break
            n *= 4
        out["cpu_baseline"] = dict(value=round(len(pix) / dt, 1), unit="rays/s",
                                   cores=int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count(),
                                   kind="oracle", sample=f"{len(pix)} rays of job 0")
    return out


# ---------------------------------------------------------------------------
# The plain single projection (one launch, one job) on the same GPU: the
# 256x256x160 ellipsoid phantom at 1.95x1.95x2.5 mm, 120 kVp + bowtie, 1e8
# photons, with the step's majorant scheme, against which the batched forward
# and the adjoint rates are read
# ---------------------------------------------------------------------------
SINGLE_PHOTONS = 100_000_000


def single_projection_leg(wl, api, W, torch, steps, fwd_rate, adj_rate):
    prob = W.pelvis_problem(SINGLE_PHOTONS)
    if SOURCE == "joint":
        prob.source = W.pelvis_source(prob.geom, joint=True)
    vol, phys, src = api.upload(prob)
    apply_majorant(vol, 2.0**-20)
    batch = api.Batch([vol], phys, [src], [api.JobSpec(prob.geom, SINGLE_PHOTONS, 0)])
    tune = autotune_for(batch)
    out = torch.zeros(batch.tally_elems, dtype=torch.float64, device="cuda")
    maj = batch.majorants(True)
    batch.project(seed=1, sumsq=False, majorants=maj, out=out, tune=tune)       # warm-up
    ms = []
    for _ in range(max(steps, 1)):
        batch.project(seed=1, sumsq=False, majorants=batch.majorants(True), out=out, tune=tune)
        ms.append(api.last_kernel_ms())
    torch.cuda.synchronize()
    kms = float(np.mean(ms))
    rate = SINGLE_PHOTONS / (kms * 1e-3)
    return dict(workload="256x256x160 @1.95x1.95x2.5mm ellipsoids, 1 angle, 1e8 photons, one launch",
                histories_per_s=round(rate, 1), transport_kernel_ms=round(kms, 3), tuning=tune,
                majorant=majorant_desc([vol]),
                batched_fwd_over_single=round(fwd_rate / rate, 4),
                adjoint_over_single=round(adj_rate / rate, 4) if adj_rate else None)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# Scatter denoising (Eq. 5) and noise assembly (Sec. 2.6) of the step's tallies
# ---------------------------------------------------------------------------
DENOISE_ITERS = 256
SLOTS_DN_SWEEP = slots(f=9, t=1)   # per pixel and sweep: 3 adds, reciprocal, mul, sub, 2 FMA, mul, max
BYTES_NOISE = 6 * 8            # Phat, P, Shat, S read; noise, image written


def denoise_leg(wl, api, torch, steps, rt_images, cpu):
    batch = wl["batch"]
    g = batch.jobs[0].geom
    if any((j.geom.nu, j.geom.nv) != (g.nu, g.nv) for j in batch.jobs):
        return None
    n = len(batch.jobs)
    tal = wl["tallies"].view(n, 4, g.nv, g.nu)
    shat = tal[:, 2]
    med = float(shat.median())
    beta = 4.0 / max(med, 1e-30)                       # beta * S ~ 4: smoothing over a few pixels
    floor = 1e-6 * max(med, 1e-30)
    p = torch.stack(rt_images) if rt_images is not None else torch.zeros(n, g.nv, g.nu, dtype=torch.float64,
                                                                             device="cuda")
    alpha = api.noise_scale(float(batch.jobs[0].n_photons), 5.2913e9, 0.6)
    api.denoise(shat, beta, DENOISE_ITERS, s_floor=floor)
    ms, wall_n = [], []
    for _ in range(max(steps, 1)):
        s_den = api.denoise(shat, beta, DENOISE_ITERS, s_floor=floor)
        ms.append(api.last_kernel_ms())
        torch.cuda.synchronize()
        t = time.perf_counter()
        api.noise(tal[:, 0], p, shat, s_den, alpha)
        torch.cuda.synchronize()
        wall_n.append((time.perf_counter() - t) * 1e3)
    kms = float(np.mean(ms))
    px = n * g.nu * g.nv
    slots = px * DENOISE_ITERS * SLOTS_DN_SWEEP / (kms * 1e-3) / 1e12
    nms = float(np.min(wall_n))
    out = dict(images=n, iters=DENOISE_ITERS, omega=0.8, beta_times_median=4.0, kernel_ms=round(kms, 3),
               pixel_sweeps_per_s=round(px * DENOISE_ITERS / (kms * 1e-3), 1),
               roofline=dict(bound="alu", achieved=round(slots, 3), peak=round(ALU_PEAK_TOPS, 2), unit="Tops/s",
                             frac=round(slots / ALU_PEAK_TOPS, 4),
                             traffic=measured_traffic(TRAFFIC_PATH, wl["config"]["workload"], "denoise")),
               noise=dict(wall_ms=round(nms, 3), alpha=round(alpha, 6),
                          roofline=dict(bound="hbm", achieved=round(px * BYTES_NOISE / (nms * 1e-3) / 1e9, 1),
                                        peak=HBM_PEAK_GBS, unit="GB/s",
                                        frac=round(px * BYTES_NOISE / (nms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                        traffic=None)))
    if cpu:
        import oracle
        img = shat[0].cpu().numpy()
        t = time.time()
        oracle.denoise(img, beta, DENOISE_ITERS, s_floor=floor)
        dt = time.time() - t
        out["cpu_baseline"] = dict(value=round(g.nu * g.nv * DENOISE_ITERS / dt, 1), unit="pixel sweeps/s",
                                   cores=1, kind="oracle", sample=f"1 image of {g.nv}x{g.nu}, {DENOISE_ITERS} sweeps")
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on a bounded sample
# ---------------------------------------------------------------------------
def cpu_baseline(wl, budget_s=20.0):
    import oracle
    oracle.build(force=False)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    stats_acc = None
    done, spent = 0, 0.0
    per = max(1, len(wl["samples"]))
    for prob, phi, jid, macro, margin, rho_min in wl["samples"]:
        p = oracle.Problem.from_workload(prob, phi_rad=phi).local_majorants(macro, margin, rho_min)
        n = 20000
        while True:                                  # grow the sample until ~budget/per seconds
            t = time.time()
            r = oracle.mc_project(p, 1, n, job_id=jid, nthreads=nthreads)
            dt = time.time() - t
            if dt > budget_s / per / 4 or n >= 1 << 24:
                break
            n *= 4
        done += n
        spent += dt
        st = r["stats"]
        if stats_acc is None:
            stats_acc = {k: (dict(v) if isinstance(v, dict) else v) for k, v in st.items()}
        else:
            for k, v in st.items():
                if isinstance(v, dict):
                    for kk, vv in v.items():
                        stats_acc[k][kk] += vv
                else:
                    stats_acc[k] += v
    fwd_rate = done / spent
    # the same jobs on one thread, about a second each: the oracle's rate per core
    done1, spent1 = 0, 0.0
    for prob, phi, jid, macro, margin, rho_min in wl["samples"]:
        p = oracle.Problem.from_workload(prob, phi_rad=phi).local_majorants(macro, margin, rho_min)
        n = 5000
        while True:
            t = time.time()
            oracle.mc_project(p, 1, n, job_id=jid, nthreads=1)
            dt = time.time() - t
            if dt > 1.0 or n >= 1 << 22:
                break
            n *= 2
        done1 += n
        spent1 += dt
    out = dict(fwd_rate=fwd_rate, fwd_sample=done, stats=stats_acc, threads=nthreads,
               fwd_rate_1=done1 / spent1, fwd_sample_1=done1)
    if wl["adjoint"] is not None:
        a = wl["adjoint"]
        p = oracle.Problem.from_workload(a["problem"]).local_majorants(a["macro"], a["margin"], a["rho_min"])
        mb = None if a["macro"] else oracle.majorant(p, True, margin=a["margin"])
        adj = np.zeros((2, p.nv, p.nu))
        adj[1] = 1.0
        n = 20000
        while True:
            t = time.time()
            oracle.mc_backward(p, 1, n, adj, mb, job_id=a["job_id"], nthreads=nthreads)
            dt = time.time() - t
            if dt > budget_s / 4 / 4 or n >= 1 << 24:
                break
            n *= 4
        out.update(adj_rate=n / dt, adj_sample=n)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-raytrace", action="store_true",
                    help="skip the ray-tracing, denoising and noise legs")
    ap.add_argument("--tune", default="auto", choices=["auto", "search", "default"],
                    help="auto: the autotuner's cached launch shape (searched if not cached); search: search "
                         "again; default: library defaults")
    ap.add_argument("--majorant", default="local", choices=["local", "global"],
                    help="local: bounds per cube of about --cube-mm (default); global: one per energy interval")
    ap.add_argument("--cube-mm", type=float, default=40.0)
    ap.add_argument("--source", default="factorised", choices=["factorised", "joint"],
                    help="factorised: one spectrum, the bowtie folded into the fluence map (default); joint: "
                         "one bowtie-hardened spectrum per detector column")
    ap.add_argument("--no-global-reference", action="store_true",
                    help="with local majorants, skip the reference forward with the single majorant")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the plain single-projection reference (one launch of 1e8 photons)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: the one shipped with the package)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="JSON with measured HBM bytes per transport launch (used if taken on this kernel)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_mib=args.calibrate_copy, read_bytes=a.numel() * 4, write_bytes=b.numel() * 4)))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path shards by job "
              f"across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    global TUNE_MODE, TUNE_CACHE, MAJORANT, CUBE_MM, TRAFFIC_PATH, SOURCE
    TUNE_MODE = args.tune
    SOURCE = args.source
    MAJORANT, CUBE_MM = args.majorant, args.cube_mm
    TRAFFIC_PATH = args.traffic
    from paper_1204_6367_amd import autotune as _at
    TUNE_CACHE = args.tune_cache or _at.DEFAULT_CACHE
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    from paper_1204_6367_amd import api, workloads as W
    api.enable_timing(True)
    t = time.time()
    wl = build_workload(args.workload, api, W, torch)
    torch.cuda.synchronize()
    log(f"setup {time.time() - t:.1f}s; fwd histories/step {wl['fwd']:.3g}, adjoint {wl['adj']:.3g}")
    for i in range(args.warmup):
        wl["step"]()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        kms.append(wl["step"]())
        log(f"step {i} done: kernel ms {kms[-1]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    hist_step = wl["fwd"] + wl["adj"]
    value = hist_step * args.steps / (t1 - t0)
    fwd_ms = float(np.mean([k[0] for k in kms]))
    adj_ms = float(np.mean([k[1] for k in kms])) if wl["adj"] else None

    glob = None
    if MAJORANT == "local" and not args.no_global_reference:
        # the same forward with one majorant per energy interval (the paper's Woodcock tracking), for reference
        b = wl["batch"]
        saved = [(v.macro, v.macro_margin, v.macro_rho_min) for v in b.vols]
        for v in b.vols:
            v.local_majorants(0)
        b.project(seed=1, sumsq=False, majorants=b.majorants(True), out=wl["tallies"])
        gms = api.last_kernel_ms()
        for v, (m, g, r) in zip(b.vols, saved):
            v.local_majorants(m, g, r)
        glob = dict(fwd_histories_per_s=round(wl["fwd"] / (gms * 1e-3), 1), transport_kernel_ms=round(gms, 3))
        log(f"global-majorant forward: {gms:.1f} ms")
    fwd_rate = wl["fwd"] / (fwd_ms * 1e-3)
    adj_rate = wl["adj"] / (adj_ms * 1e-3) if adj_ms else None
    single = None
    if not args.no_single:
        single = single_projection_leg(wl, api, W, torch, args.steps, fwd_rate, adj_rate)
        log(f"single projection: {single['transport_kernel_ms']:.2f} ms, {single['histories_per_s']:.4g} histories/s")
    rt = None if args.no_raytrace else raytrace_leg(wl, api, torch, args.steps, not args.no_cpu_baseline)
    dn = None if args.no_raytrace else denoise_leg(wl, api, torch, args.steps, wl["batch"].primary(),
                                                   not args.no_cpu_baseline)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)
    roof = None
    extra = {}
    if cpu is not None:
        w = work_per_history(cpu["stats"], cpu["fwd_sample"])
        slots = w["slots"] * wl["fwd"]
        nbytes = w["bytes"] * wl["fwd"]
        alu_ach = slots / (fwd_ms * 1e-3) / 1e12
        hbm_ach = nbytes / (fwd_ms * 1e-3) / 1e9
        traffic = measured_traffic(args.traffic, args.workload)
        alu = dict(bound="alu", achieved=round(alu_ach, 3), peak=round(ALU_PEAK_TOPS, 2), unit="Tops/s",
                   frac=round(alu_ach / ALU_PEAK_TOPS, 4), traffic=traffic)
        hbm = dict(bound="hbm", achieved=round(hbm_ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(hbm_ach / HBM_PEAK_GBS, 4), traffic=traffic)
        roof = alu if alu["frac"] >= hbm["frac"] else hbm
        extra["roofline_other"] = hbm if roof is alu else alu
        extra["work_per_history"] = {k: round(v, 3) for k, v in w.items()}
        rg = gather_roofline(GATHER_PATH, wl["batch"], w["inbox_flights"], wl["fwd"] / (fwd_ms * 1e-3))
        if rg is not None:
            extra["roofline_gather"] = rg
        cores = cpu["threads"]
        if wl["adj"]:
            cval = hist_step / (wl["fwd"] / cpu["fwd_rate"] + wl["adj"] / cpu["adj_rate"])
            sample = (f"{cpu['fwd_sample']} forward histories over {len(wl['samples'])} jobs + "
                      f"{cpu['adj_sample']} adjoint histories of the same workload")
        else:
            cval = cpu["fwd_rate"]
            sample = f"{cpu['fwd_sample']} forward histories over {len(wl['samples'])} jobs of the same workload"
        cpu = dict(value=round(cval, 1), unit="histories/s", cores=cores, cpu_model=cpu_model(), kind="oracle",
                   sample=sample,
                   single_thread=dict(value=round(cpu["fwd_rate_1"], 1), unit="forward histories/s", cores=1,
                                      sample=f"{cpu['fwd_sample_1']} forward histories over {len(wl['samples'])} jobs"))
    line = dict(metric=METRIC, value=round(value, 1), unit="histories/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(ms_step, 2), higher_is_better=True, scaling="weak",
                vs_baseline=None, dtype="f32", data="synthetic",
                config=wl["config"], roofline=roof, cpu_baseline=cpu,
                counters=measured_counters(args.traffic, args.workload),
                adjoint_counters=measured_counters(args.traffic, args.workload, "adjoint") if wl["adj"] else None,
                fwd_histories_per_s=round(fwd_rate, 1),
                adj_histories_per_s=round(adj_rate, 1) if adj_rate else None,
                single_projection=single,
                transport_kernel_ms=round(fwd_ms, 3), adjoint_kernel_ms=round(adj_ms, 3) if adj_ms else None,
                **extra, global_majorant=glob, raytrace=rt, denoise=dn)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
