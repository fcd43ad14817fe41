"""Pins for the selector-feature oracle (oracle/features.py) on inputs whose
features have closed forms."""
import math

import numpy as np

from oracle import features as F


def test_constant_edges():
    m, n = 5000, 1000
    z = np.zeros(m, np.int64)
    f = F.features(z, z, n)
    assert f[0] == math.log2(1 + n) and f[1] == math.log2(1 + m)
    assert math.isclose(f[2], math.log2(1 + m / n))
    assert math.isclose(f[3], math.log2(1 + n))          # every pair collides
    assert math.isclose(f[4], math.log2(1 + n))
    assert math.isclose(f[5], math.log2(1 + n))          # one value, K times
    assert math.isclose(f[6], math.log2(1 + n))
    assert f[7] == 1 / F.K_SPREAD and f[8] == 1 / F.K_SPREAD
    assert f[9] == 0.0                                   # src == dst
    assert f[10] == 1 / 1024 and f[11] == 1 / 1024       # one cache line per window
    assert f[12] == 1.0 and f[14] == 1.0                 # all neighbours equal
    assert f[13] == 1.0 and f[15] == 1.0


def test_constant_destination_distinct_sources():
    # dst constant, src = e: only the destination side is concentrated, so
    # every dst-side feature takes its all-equal value and every src-side one
    # its all-distinct value (this separates f[6] from f[5])
    m = 64 * 1024
    n = m
    src = np.arange(m, dtype=np.int64)
    dst = np.full(m, 7, np.int64)
    f = F.features(src, dst, n)
    assert math.isclose(f[6], math.log2(1 + n))          # maxcount_dst = K
    assert math.isclose(f[5], math.log2(1 + n / F.K_SPREAD))  # maxcount_src = 1
    assert math.isclose(f[4], math.log2(1 + n)) and f[3] == 0.0
    assert f[8] == 1 / F.K_SPREAD and f[7] == 1.0
    assert f[13] == 1.0 and f[12] == 0.0
    assert f[11] == 1 / 1024 and math.isclose(f[10], 32 / 1024)


def test_grouped_sources_aligned_windows():
    # src = e // 4, 64 windows of 1024 starting at multiples of 1024
    m = 64 * 1024
    e = np.arange(m, dtype=np.int64)
    src = e // 4
    dst = e
    n = m
    f = F.features(src, dst, n)
    assert math.isclose(f[12], 768 / 1023)              # 3 equal pairs per group of 4
    assert f[13] == 0.0
    assert f[14] == 1.0 and f[15] == 1.0                # consecutive steps of 0 or 1
    assert math.isclose(f[10], 8 / 1024)                # 256 sources span 8 lines of 32
    assert math.isclose(f[11], 32 / 1024)               # 1024 destinations span 32 lines
    # |src - dst| = e - e//4 summed per window
    expect = np.mean([(e[s:s + 1024] - src[s:s + 1024]).sum() / (1024 * n) for s in range(0, m, 1024)])
    assert math.isclose(f[9], expect, rel_tol=1e-12)
    # spread samples: k*16; sources k*4 are distinct, as are destinations
    assert f[7] == 1.0 and f[8] == 1.0 and f[3] == 0.0 and f[4] == 0.0
    assert math.isclose(f[5], math.log2(1 + n / F.K_SPREAD))


def test_empty_and_tiny():
    f = F.features(np.zeros(0, np.int64), np.zeros(0, np.int64), 10)
    assert np.count_nonzero(f[3:]) == 0 and f[0] == math.log2(11)
    f = F.features(np.array([3]), np.array([5]), 10)
    assert f[12] == 0.0 and f[7] == 1 / F.K_SPREAD     # one edge sampled K times... as one value
    assert math.isclose(f[9], 2 / 10)
