"""Pins for the oracle's random-number and Gaussian arithmetic.

These check the oracle against things other than itself: the published
Philox4x32-10 known-answer vectors, the open-source rocRAND implementation of
the same bijection (compiled for the host, test only), the exact values of
ln/sin/cos over every reachable input, the Gaussian law of the Box-Muller
output, and the statistics of the quarter-disc estimate of pi that the paper
uses to compare generators (Sec. 3, Table rngs).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    for ctr, key, out in _kat():
        got = oracle_lib.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == out


_ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // reads lines "c01(64-bit) c23(64-bit) seed(64-bit)" and prints four words
  unsigned long long c01, c23, seed;
  while (std::scanf("%llx %llx %llx", &c01, &c23, &seed) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, c23, 4ull * c01);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_host(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "ref.hip"
    src.write_text(_ROCRAND_SRC)
    exe = d / "ref"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", str(exe), str(src)],
                   check=True, capture_output=True)
    return str(exe)


def test_philox_matches_rocrand_host(oracle_lib, rocrand_host):
    rng = np.random.default_rng(7)
    lines, expect = [], []
    for _ in range(2000):
        c = rng.integers(0, 2**32, 4, dtype=np.uint64)
        c[1] &= 0x3FFFFFFF  # the engine takes words 0-1 as an offset of 4 * c01 numbers
        s = int(rng.integers(0, 2**63, dtype=np.uint64)) * 2 + int(rng.integers(0, 2))
        c01 = int(c[0]) | (int(c[1]) << 32)
        c23 = int(c[2]) | (int(c[3]) << 32)
        lines.append(f"{c01:x} {c23:x} {s:x}")
        key = [s & 0xFFFFFFFF, s >> 32]
        expect.append(oracle_lib.philox4x32_10([int(x) for x in c], key))
    out = subprocess.run([rocrand_host], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for e, o in zip(expect, out):
        assert [int(t, 16) for t in o.split()] == [int(x) for x in e]


def _ulp32(x):
    x = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.maximum(x, 2.0**-126)))
    return 2.0 ** (e - 23)


def test_ln_every_input(oracle_lib):
    """ln(K 2^-24) over all 2^24 inputs: within 2 ulp of the exact value."""
    K = np.arange(1, 2**24 + 1, dtype=np.float64)
    got = oracle_lib.ln_u24_bulk(1, 2**24).astype(np.float64)
    exact = np.log(K) - 24.0 * math.log(2.0)
    err = np.abs(got - exact)
    nz = exact != 0.0
    assert got[-1] == 0.0 and exact[-1] == 0.0
    ulps = err[nz] / _ulp32(exact[nz])
    assert ulps.max() <= 2.0, ulps.max()
    # monotone non-decreasing in K, as ln is
    assert np.all(np.diff(got) >= 0.0)


def test_sincos_every_input(oracle_lib):
    """sin and cos of 2 pi J 2^-24 over all 2^24 inputs: absolute error
    below 2^-23 and the Pythagorean identity within 4 * 2^-24 (two
    errors of about one ulp of 1/sqrt(2), each doubled by the square)."""
    s, c = oracle_lib.sincos_bulk(0, 2**24)
    th = 2.0 * np.pi * np.arange(2**24, dtype=np.float64) / 2**24
    es = np.abs(s.astype(np.float64) - np.sin(th))
    ec = np.abs(c.astype(np.float64) - np.cos(th))
    assert es.max() < 2.0**-23 and ec.max() < 2.0**-23, (es.max(), ec.max())
    # small angles keep relative accuracy (no cancellation near the axes)
    small = (np.abs(np.sin(th)) > 2.0**-20)
    assert (es[small] / _ulp32(np.sin(th[small]))).max() <= 4.0
    pyth = np.abs(s.astype(np.float64) ** 2 + c.astype(np.float64) ** 2 - 1.0)
    assert pyth.max() < 4 * 2.0**-24
    # quarter-turn symmetries are exact: sin(t + pi/2) = cos(t)
    q = 2**22
    assert np.array_equal(s[q:2 * q], c[0:q])
    assert np.array_equal(c[q:2 * q], -s[0:q])


def test_box_muller_is_standard_normal(oracle_lib):
    rng = np.random.default_rng(11)
    n = 1_000_000
    ra = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    rb = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    z0, z1 = oracle_lib.box_muller_bulk(ra, rb)
    for z in (z0, z1):
        z = z.astype(np.float64)
        assert abs(z.mean()) < 5.0 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert abs(stats.skew(z)) < 5.0 * math.sqrt(6.0 / n)
        assert abs(stats.kurtosis(z)) < 5.0 * math.sqrt(24.0 / n)
        assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 5.0 / math.sqrt(n)
    # radius law: z0^2 + z1^2 ~ chi^2_2 = Exp(mean 2)
    r2 = z0.astype(np.float64) ** 2 + z1.astype(np.float64) ** 2
    assert stats.kstest(r2, "expon", args=(0, 2.0)).pvalue > 1e-4


def test_box_muller_extremes(oracle_lib):
    # u_a = 2^-24 (ra>>8 = 0) gives the largest radius sqrt(48 ln 2)
    z0, z1 = oracle_lib.box_muller(0, 0)
    assert abs(float(z0) - math.sqrt(48.0 * math.log(2.0))) < 1e-6 and z1 == 0.0
    # u_a = 1 gives radius 0
    z0, z1 = oracle_lib.box_muller(0xFFFFFFFF, 12345 << 8)
    assert z0 == 0.0 and z1 == 0.0


def test_pi_estimate_statistics(oracle_lib):
    """Quarter-disc estimator of pi (Sec. 3, Table rngs).  The paper's
    printed standard deviations for 500 repetitions of 1e9 points
    (5.26e-5, 5.21e-5, 5.03e-5) match 4 sqrt(p(1-p)/M), p = pi/4, with M
    counting points; the same law must hold for Philox uniforms at a
    size the CPU finishes quickly."""
    p = math.pi / 4.0
    theory_paper = 4.0 * math.sqrt(p * (1 - p) / 1e9)
    for printed in (5.2585e-05, 5.20932e-05, 5.03272e-05):
        assert abs(printed / theory_paper - 1.0) < 0.05
    reps, M = 100, 2_000_000
    est = np.array([oracle_lib.pi_estimate(0x5EED0000, r, M) for r in range(reps)])
    sd = 4.0 * math.sqrt(p * (1 - p) / M)
    assert abs(est.mean() - math.pi) < 4.0 * sd / math.sqrt(reps)
    # sample std within the 99.99% chi-square band for 99 degrees of freedom
    lo, hi = stats.chi2.ppf([1e-4, 1 - 1e-4], reps - 1)
    s2 = est.var(ddof=1)
    assert lo / (reps - 1) < s2 / sd**2 < hi / (reps - 1)
