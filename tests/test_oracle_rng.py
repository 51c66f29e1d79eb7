"""Pins for the oracle's random-number layer (not the GPU).

Philox4x32-10 (Salmon et al., SC'11) is checked word for word against an
independent implementation, rocRAND's header-only engine evaluated on the
host.  The uniform, Box-Muller normal and Marsaglia-Tsang Gamma layers are
checked against their laws with scipy.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("probe") / "rprobe")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_probe.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(12345)
    rows = []
    edge = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF]
    for e in edge:
        rows.append((e | (e << 32), e, e, e, e))
    for _ in range(300):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        c = [int(v) for v in rng.integers(0, 2 ** 32, size=4)]
        rows.append((seed, *c))
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        seed, c0, c1, c2, c3 = r
        ref = [int(v) for v in line.split()]
        got = orc.philox([c0, c1, c2, c3], [seed & 0xFFFFFFFF, seed >> 32])
        assert list(map(int, got)) == ref, (r, got, ref)


def test_philox_words_uniform(orc):
    # chi-square on the top byte of 4 x 20000 words from consecutive counters
    words = np.concatenate([orc.philox([i, 3, 1, 0], [7, 9]) for i in range(20000)])
    top = (words >> 24).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4


def test_uniform52_open_interval(orc):
    lo = orc.uniform52(0, 0)
    hi = orc.uniform52(0xFFFFFFFF, 0xFFFFFFFF)
    assert lo == 0.5 * 2.0 ** -52
    assert hi == 1.0 - 0.5 * 2.0 ** -52
    assert 0.0 < lo < hi < 1.0
    # the top 52 bits are used: the low 12 bits of the second word are ignored
    assert orc.uniform52(5, 0xFFF) == orc.uniform52(5, 0)
    assert orc.uniform52(5, 0x1000) > orc.uniform52(5, 0xFFF)
    assert orc.uniform52(1, 0) == (2.0 ** 20 + 0.5) * 2.0 ** -52


def test_normal_law(orc):
    z = orc.site_normals(seed=2024, sweep=3, instance=1, n=200000)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 0.05
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_normal_is_box_muller_of_block(orc):
    # z = sqrt(-2 ln u1) cos(2 pi u2) with (u1, u2) from the words of the block
    for (seed, c) in [(1, (0, 0, 0, 0)), (99, (17, 4, 2, 0)), (2 ** 40 + 3, (5, 1, 0, 0))]:
        w = orc.philox(list(c), [seed & 0xFFFFFFFF, seed >> 32])
        u1 = orc.uniform52(int(w[0]), int(w[1]))
        u2 = orc.uniform52(int(w[2]), int(w[3]))
        ref = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        assert abs(orc.normal(seed, *c) - ref) <= 1e-15 * max(1.0, abs(ref))


def test_streams_do_not_collide(orc):
    # site normals of different sweeps / instances / tags are different draws
    a = orc.normal(5, 10, 0, 0, 0)
    assert a != orc.normal(5, 10, 1, 0, 0)
    assert a != orc.normal(5, 10, 0, 1, 0)
    assert a != orc.normal(5, 10, 0, 0, 1)
    assert a != orc.normal(6, 10, 0, 0, 0)


@pytest.mark.parametrize("shape", [1.0, 2.5, 2048.5, 2.1e6])
def test_gamma_law(orc, shape):
    rate = 3.0
    N = 20000
    draws = np.empty(N)
    for t in range(N):
        v, a = orc.gamma(shape, rate, seed=77, sweep=t, instance=0, tag=1)
        assert a >= 1
        draws[t] = v
    mean, var = shape / rate, shape / rate ** 2
    assert abs(draws.mean() - mean) < 5 * np.sqrt(var / N)
    assert abs(draws.var() / var - 1.0) < 5 * np.sqrt(2.0 / N) * (1 + 3 / shape)
    p = stats.kstest(draws, stats.gamma(shape, scale=1.0 / rate).cdf).pvalue
    assert p > 1e-4


def test_gamma_acceptance_and_errors(orc):
    # Marsaglia-Tsang accepts with probability > 0.95 for shape >= 1
    attempts = [orc.gamma(1.0, 1.0, 3, t, 0, 2)[1] for t in range(5000)]
    assert np.mean(attempts) < 1.06
    with pytest.raises(ValueError):
        orc.gamma(0.5, 1.0, 1, 0, 0, 1)
    with pytest.raises(ValueError):
        orc.gamma(2.0, 0.0, 1, 0, 0, 1)
    # attempt cap 0 always fails (the device status path relies on this)
    v, a = orc.gamma(2.0, 1.0, 1, 0, 0, 1, max_attempts=0)
    assert a == -1 and np.isnan(v)


def test_gamma_scales_with_rate(orc):
    # same counters, same shape: the draw is d*v/rate, so it scales as 1/rate
    v1, _ = orc.gamma(10.0, 1.0, 11, 4, 2, 1)
    v2, _ = orc.gamma(10.0, 4.0, 11, 4, 2, 1)
    assert abs(v1 / 4.0 - v2) <= 1e-15 * v1
