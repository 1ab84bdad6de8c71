"""Host-side logic of the benchmark (CPU only): the one-GPU guard, the
measured-traffic records (used only while they match the kernel sources),
and the per-history work model built from the oracle's counts."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_follows_the_kernel_sources(tmp_path):
    sha = bench.kernel_sources_sha()
    rec = {"c4": {"kernel_sha": sha, "fetch_bytes": 1000, "write_bytes": 24,
                  "others": {"raytrace": {"fetch_bytes": 7, "write_bytes": 3}}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(str(p), "c4") == 1024
    assert bench.measured_traffic(str(p), "c4", "raytrace") == 10
    assert bench.measured_traffic(str(p), "c4", "denoise") is None
    assert bench.measured_traffic(str(p), "c1") is None
    rec["c4"]["kernel_sha"] = "0" * 16                     # taken on other sources: not used
    p.write_text(json.dumps(rec))
    assert bench.measured_traffic(str(p), "c4") is None
    assert bench.measured_traffic(str(tmp_path / "missing.json"), "c4") is None
    p.write_text("not json")
    assert bench.measured_traffic(str(p), "c4") is None


def test_shipped_traffic_record_names_its_summary():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["c4"]
    assert os.path.exists(os.path.join(ROOT, rec["summary"]))
    assert rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
    assert set(rec["others"]) == {"raytrace", "denoise", "adjoint"}
    # the counter readings the benchmark line carries
    c = rec["counters"]
    assert 0.0 < c["lanes_active"] <= 1.0 and 0.0 < c["l2_hit"] < 1.0
    lo, hi = c["valu_issue_util"]
    assert 0.0 < lo <= hi <= 1.0


def test_measured_counters_follow_the_kernel_sources(tmp_path):
    sha = bench.kernel_sources_sha()
    ctr = {"lanes_active": 0.3, "valu_inst_rate": 1.05, "valu_issue_util": [0.8, 1.0], "l2_hit": 0.45,
           "duration_ms": 3.0}
    rec = {"c4": {"kernel": "k", "kernel_sha": sha, "counters": ctr,
                  "others": {"adjoint": {"kernel": "a", "counters": dict(ctr, lanes_active=0.2)}}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(rec))
    got = bench.measured_counters(str(p), "c4")
    assert got["lanes_active"] == 0.3 and got["kernel"] == "k" and "duration_ms" not in got
    assert bench.measured_counters(str(p), "c4", "adjoint")["lanes_active"] == 0.2
    assert bench.measured_counters(str(p), "c4", "raytrace") is None
    rec["c4"]["kernel_sha"] = "0" * 16
    p.write_text(json.dumps(rec))
    assert bench.measured_counters(str(p), "c4") is None


def test_work_model_composition():
    """Slots and bytes per history add up from the oracle's counts as stated."""
    n = 1000
    stats = dict(steps=7000.0, real=2500.0, tries=2900.0, compton=2000.0, rayleigh=100.0, crossings=11000.0,
                 classes=dict(primary=3.0, scatter=2.0, absorbed=600.0, cut=0.0, missed=395.0, lost=0.0))
    w = bench.work_per_history(stats, n)
    assert w["flights"] == pytest.approx(7.0)
    assert w["inbox_flights"] == pytest.approx(7.0 - 0.4)
    assert w["cube_visits"] == pytest.approx(11.0 + 7.0)
    pairs = 0.5 * (7.0 + 2.5)
    base = (pairs * bench.SLOTS_PHILOX + 6.6 * bench.SLOTS_FLIGHT_IN + 0.4 * bench.SLOTS_FLIGHT_OUT
            + 2.9 * bench.SLOTS_TRY + 2.5 * bench.SLOTS_SELECT + 2.1 * (bench.SLOTS_COLLISION - bench.SLOTS_SELECT)
            + bench.SLOTS_SOURCE)
    # local majorants: a walk set-up per pair of flights and the cube visits, no box exit after a collision
    assert w["slots"] == pytest.approx(base + pairs * bench.SLOTS_WALK + 18.0 * bench.SLOTS_CUBE)
    nbytes = 6.6 * bench.BYTES_FLIGHT_IN + bench.BYTES_SOURCE + 0.005 * bench.BYTES_SCORE + 18.0 * bench.BYTES_CUBE
    assert w["bytes"] == pytest.approx(nbytes)
    # the single majorant: no cube walk, and every scattering recomputes the distance to the box
    stats["crossings"] = 0.0
    w0 = bench.work_per_history(stats, n)
    assert w0["cube_visits"] == 0.0
    assert w0["slots"] == pytest.approx(base + 2.1 * bench.SLOTS_BOX_EXIT)


def test_work_model_prices_measured_issue_costs():
    """Instruction classes at the costs the calibration program measures on
    gfx950, in slots of a full-rate integer operation: integer operations and
    32x32-bit products 1, float32 arithmetic with vector operands 0.6,
    transcendentals 2.3.  A Philox4x32-10 block is ten rounds of two products
    and two three-input xors (v_bitop3_b32)."""
    assert (bench.SLOTS_INT, bench.SLOTS_F32, bench.SLOTS_TRANS) == (1.0, 0.6, 2.3)
    assert bench.slots(i=3, f=5, t=2) == pytest.approx(3 + 3.0 + 4.6)
    assert bench.SLOTS_PHILOX == 40
    assert bench.SLOTS_DN_SWEEP == pytest.approx(9 * 0.6 + 2.3)
    assert bench.SLOTS_RT_INTERVAL == pytest.approx(13 + 33 * 0.6)


def test_gather_roofline_from_measured_rates(tmp_path):
    """The transport's gather roofline: one 32-byte cell record per free flight
    inside a phantom, against the random-gather rate measured at the smallest
    working set that holds each phantom's cell records, the rates combined
    harmonically by photons."""
    import types
    rates = {"32": [[1 << 21, 8000.0], [1 << 27, 2000.0], [1 << 32, 1500.0]]}
    p = tmp_path / "g.json"
    p.write_text(json.dumps({"rates": rates}))
    assert bench.gather_peak(rates["32"], 1 << 20) == 8000.0
    assert bench.gather_peak(rates["32"], (1 << 21) + 1) == 2000.0
    assert bench.gather_peak(rates["32"], 1 << 40) == 1500.0
    vol = lambda shape: types.SimpleNamespace(density=types.SimpleNamespace(shape=shape))
    job = lambda v, n: types.SimpleNamespace(volume=v, n_photons=n)
    # cell records: 9x9x9 x 32 B (23 KB, within 2 MiB) and 257^3 x 32 B (543 MB, beyond 128 MiB)
    b = types.SimpleNamespace(vols=[vol((8, 8, 8)), vol((256, 256, 256))], jobs=[job(0, 300), job(1, 100)])
    r = bench.gather_roofline(str(p), b, inbox_flights=5.0, histories_per_s=1e9)
    peak = 1.0 / (0.75 / 8000.0 + 0.25 / 1500.0)
    assert r["peak"] == pytest.approx(peak, abs=0.1)
    assert r["achieved"] == pytest.approx(5.0 * 32 * 1e9 / 1e9)
    assert r["frac"] == pytest.approx(160.0 / peak, abs=1e-4)
    assert bench.gather_roofline(str(tmp_path / "missing.json"), b, 5.0, 1e9) is None
