"""Pins of the oracle's random-number layer: Philox4x32-10 and the samplers of
tabulated pdfs.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle_lib.philox(ctr, key)
        assert [int(x) for x in got] == want


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
    // args: seed subsequence offset  -> prints the four words of that block
    unsigned long long seed = strtoull(argv[1], 0, 0), sub = strtoull(argv[2], 0, 0), off = strtoull(argv[3], 0, 0);
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_header(oracle_lib, tmp_path):
    """Independent implementation: rocRAND's open-source header, built for the
    host.  Its engine keys with the 64-bit seed and puts (offset/4) in counter
    words 0-1 and the subsequence in words 2-3."""
    src = tmp_path / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = tmp_path / "probe"
    r = subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                        str(src), "-o", str(exe)], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND probe: " + r.stderr[-400:])
    rng = np.random.default_rng(7)
    for _ in range(6):
        c = [int(x) for x in rng.integers(0, 2**32, 4)]
        c[1] &= (1 << 29) - 1                       # keep 4*offset inside 64 bits
        k = [int(x) for x in rng.integers(0, 2**32, 2)]
        seed = k[0] | (k[1] << 32)
        sub = c[2] | (c[3] << 32)
        off = 4 * (c[0] | (c[1] << 32))
        out = subprocess.run([str(exe), str(seed), str(sub), str(off)], capture_output=True,
                             text=True, timeout=60, check=True).stdout.split()
        assert [int(x) for x in out] == [int(x) for x in oracle_lib.philox(c, k)]


def test_philox_words_look_uniform(oracle_lib):
    """Bit balance and a KS test of u24 over a counter sweep (sanity, not a pin)."""
    from scipy import stats
    words = np.array([oracle_lib.philox([i, 3, 1, 0], [1, 0]) for i in range(4000)], np.uint64)
    bits = ((words[..., None] >> np.arange(32, dtype=np.uint64)) & 1).mean(axis=(0, 1))
    assert np.all(np.abs(bits - 0.5) < 0.02)
    u = ((words.ravel() >> 9).astype(np.float64) + 0.5) / 2**23
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_inverse_cdf_matches_searchsorted(oracle_lib):
    """Smallest k with u < C_k, C = cumsum / total (numpy's own routines)."""
    rng = np.random.default_rng(3)
    w = rng.random(1000).astype(np.float32)
    w[rng.random(1000) < 0.2] = 0.0                 # empty bins must never be drawn
    u = np.concatenate([rng.random(200000), [0.0, 1.0 - 2**-53]])
    got = oracle_lib.sample_cdf(w, u)
    cdf = np.cumsum(w.astype(np.float64))
    cdf = cdf / cdf[-1]
    want = np.searchsorted(cdf, u, side="right")
    assert np.array_equal(got, want)
    assert np.all(w[got] > 0)


def test_inverse_cdf_frequencies(oracle_lib):
    from scipy import stats
    w = np.array([0.1, 0.0, 0.3, 0.05, 0.55], np.float32)
    u = np.random.default_rng(4).random(400000)
    k = oracle_lib.sample_cdf(w, u)
    counts = np.bincount(k, minlength=5)
    assert counts[1] == 0
    nz = w > 0
    exp = w[nz] / w.sum() * len(u)
    assert stats.chisquare(counts[nz], exp).pvalue > 1e-4


def test_inverse_cdf_rejects_bad_weights(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.sample_cdf(np.array([0.0, 0.0], np.float32), np.array([0.5]))
    with pytest.raises(ValueError):
        oracle_lib.sample_cdf(np.array([1.0, -1.0], np.float32), np.array([0.5]))
