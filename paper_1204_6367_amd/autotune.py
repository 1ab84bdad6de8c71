"""Launch-shape autotuner for the persistent transport kernel.

Times candidate launch shapes (workgroup size, refill and collision
deferral, then chunk size and workgroups per CU) on a reduced copy of a batch
(same phantoms, sources and angles, a fraction of the photons) with the
library's kernel timing hook, and caches the fastest per workload class, mode,
kernel-source hash and device in a JSON file.  Tallies do not depend on the shape (integer tallies keyed by
photon index), so tuning never changes results.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
from typing import Dict, Iterable, List, Optional

import torch

from . import api

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

# Stage 1: block x refill deferral x collision deferral; stage 2, one field at a
# time from the best so far: chunk size, workgroups per CU.
CANDIDATES: List[Dict[str, int]] = [
    dict(block=b, defer=d, coll_defer=c, chunk=0, blocks_per_cu=0)
    for b in (256, 512, 1024) for d in (8, 16, 24, 32) for c in (0, 12, 20, 28)
]
REFINE: List[Dict[str, int]] = [dict(chunk=c) for c in (128, 512, 2048)] + [dict(blocks_per_cu=n) for n in (1, 2, 3, 4)]


def kernel_sha() -> str:
    """Hash of the HIP sources: a cached shape is valid only for the kernels it was timed on."""
    h = hashlib.sha1()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def workload_key(batch: "api.Batch", mode: str = "forward", interp: bool = True) -> str:
    vols = ";".join("x".join(map(str, v.shape)) + (f"/m{v.macro}" if v.macro else "") for v in batch.vols)
    dets = sorted({(j.geom.nu, j.geom.nv) for j in batch.jobs})
    # the architecture and CU count, not the marketing name (which depends on the host's ids file)
    if torch.cuda.is_available():
        pr = torch.cuda.get_device_properties(torch.cuda.current_device())
        dev = f"{pr.gcnArchName.split(':')[0]}/{pr.multi_processor_count}cu"
    else:
        dev = "cpu"
    return (f"vols={vols}|det={dets}|jobs={len(batch.jobs)}|mode={mode}|interp={int(interp)}"
            f"|src={kernel_sha()}|dev={dev}")


def _reduced(batch: "api.Batch", fraction: float, min_photons: int) -> "api.Batch":
    jobs = [api.JobSpec(j.geom, max(min_photons, int(j.n_photons * fraction)), j.job_id, j.volume, j.source)
            for j in batch.jobs]
    return api.Batch(batch.vols, batch.phys, batch.srcs, jobs)


def autotune(batch: "api.Batch", candidates: Optional[Iterable[Dict[str, int]]] = None,
             fraction: float = 0.05, min_photons: int = 100_000, repeats: int = 2,
             cache: Optional[str] = DEFAULT_CACHE, force: bool = False, interp: bool = True,
             mode: str = "forward", volume: int = 0) -> Dict[str, int]:
    """Returns the fastest tuning dict for `batch` (cached by workload class).
    mode "backward" times the adjoint of `volume` (adjoint weights 1 on the
    scatter images, so that every scored scatter history is replayed)."""
    if mode not in ("forward", "backward"):
        raise ValueError("mode must be 'forward' or 'backward'")
    key = workload_key(batch, mode, interp)
    table = {}
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
    if not force and key in table:
        return dict(table[key]["tuning"])
    if not force:
        print(f"autotune: no cached shape for {key} in {cache}", file=sys.stderr, flush=True)
    small = _reduced(batch, fraction, min_photons)
    maj = small.majorants(interp)
    adj = None
    if mode == "backward":
        g = small.jobs[0].geom
        adj = torch.zeros(len(small.jobs), 2, g.nv, g.nu, dtype=torch.float64, device=maj.device)
        adj[:, 1] = 1.0
    api.enable_timing(True)
    results = []

    def run(cand):
        try:
            _timed(small, maj, cand, interp, adj, volume)                 # warm-up / graph build
            ms = min(_timed(small, maj, cand, interp, adj, volume) for _ in range(repeats))
        except api._abi.GdrrError:
            return
        results.append((ms, cand))

    for cand in (candidates or CANDIDATES):
        run(dict(cand))
    if not results:
        raise RuntimeError("no candidate launch shape ran")
    if candidates is None:                      # refine one field at a time from the best so far
        for r in REFINE:
            best = min(results, key=lambda x: x[0])[1]
            if all(best.get(k) == v for k, v in r.items()):
                continue
            run({**best, **r})
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    if cache:
        table[key] = dict(tuning=best, ms=best_ms, photons=sum(j.n_photons for j in small.jobs),
                          all=[dict(ms=m, **c) for m, c in results])
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, cache)
    return dict(best)


def _timed(batch, maj, cand, interp, adj=None, volume=0) -> float:
    if adj is None:
        batch.project(seed=1, interp=interp, sumsq=False, majorants=maj, tune=cand)
    else:
        batch.backward(adj, maj, volume=volume, seed=1, interp=interp, tune=cand)
    return api.last_kernel_ms()
