"""Pins of the oracle's random-number pieces against things other than itself.

* Philox4x32-10 block function: compared with rocRAND's independent
  implementation (open-source headers, compiled here for the host).
* rand(N) of Sec. 2.1: the map floor(x*N/2^32) is monotone, so checking every
  bucket boundary (computed with exact Python integers) fixes it completely.
* Weight transforms: closed-form special cases and distribution tests.
* ms -> step delay conversion (Sec. 2.1): hand-checkable cases, ties to even.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("probe") / "probe")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_probe.cpp")],
                   check=True, capture_output=True)
    return exe


def _rocrand_words(exe, seed, sub, off, n):
    out = subprocess.run([exe, str(seed), str(sub), str(off), str(n)], check=True,
                         capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("seed,c,s,q0", [
    (0, 0, 0, 0),
    (12345, 0, 0, 0),
    (12345, 3, 0, 4 * 1000),
    (12345, 3, 1, 4 * 77),
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 1, 4 * (2**32 + 5)),
    (0xFFFFFFFFFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 4 * (2**61)),
    (0x0123456789ABCDEF, 4095, 0, 4 * 123456789),
])
def test_philox_matches_rocrand(rocrand_probe, seed, c, s, q0):
    # rocRAND's engine takes (seed, subsequence, offset); our word stream is
    # keyed by seed with counter (q/4, c, s): subsequence = c | s << 32.
    n = 64
    ref = _rocrand_words(rocrand_probe, seed, c | (s << 32), q0, n)
    got = [oracle.word(seed, c, s, q0 + k) for k in range(n)]
    assert got == ref


def test_philox_block_function_direct(rocrand_probe):
    # The block function with an arbitrary 128-bit counter and 64-bit key.
    for ctr, key in [((1, 2, 3, 4), (5, 6)),
                     # rocRAND's offset is a 64-bit word count, so the counter's
                     # second word stays below 2^30 here
                     ((0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF)),
                     ((0x243F6A88, 0x05A308D3, 0x13198A2E, 0x83707344), (0xA4093822, 0x299F31D0))]:
        seed = key[0] | (key[1] << 32)
        sub = ctr[2] | (ctr[3] << 32)
        off = 4 * (ctr[0] | (ctr[1] << 32))
        assert oracle.philox(ctr, key) == _rocrand_words(rocrand_probe, seed, sub, off, 4)


def test_philox_bit_balance():
    words = np.array([oracle.word(99, 1, 0, q) for q in range(1 << 14)], dtype=np.uint64)
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).sum(axis=0)
    n = words.size
    # each bit is a fair coin: |count - n/2| < 5 sigma
    assert np.all(np.abs(bits - n / 2) < 5 * np.sqrt(n / 4))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 20, 1000, 77169, 1_000_000, 2**31 + 1, 2**32 - 1])
def test_rand_below_bucket_boundaries(n):
    # R(x, n) = floor(x n / 2^32) is non-decreasing in x.  The smallest x with
    # R(x) = y is b_y = ceil(y 2^32 / n); checking R(b_y) = y and R(b_y - 1) = y - 1
    # for every bucket pins the whole map.  Buckets of large n are sampled.
    ys = np.arange(1, n, dtype=np.int64) if n <= 200_000 else np.unique(
        np.concatenate([np.arange(1, 1000), np.random.default_rng(n % 1000).integers(1, n, 20000),
                        np.arange(n - 1000, n)]))
    b = np.array([-(-int(y) * 2**32 // n) for y in ys], dtype=np.uint64)
    at = oracle.rand_below(b.astype(np.uint32), n)
    before = oracle.rand_below((b - 1).astype(np.uint32), n)
    assert np.array_equal(at.astype(np.int64), ys)
    assert np.array_equal(before.astype(np.int64), ys - 1)
    assert oracle.rand_below(np.array([0], np.uint32), n)[0] == 0
    assert oracle.rand_below(np.array([2**32 - 1], np.uint32), n)[0] == n - 1
    # preimage sizes are floor or ceil of 2^32 / n
    if n <= 200_000:
        full = np.concatenate([[0], b, [2**32]]).astype(np.float64)
        sizes = np.diff(full)
        assert set(np.unique(sizes)) <= {2**32 // n, -(-(2**32) // n)}


# --- weight transforms ----------------------------------------------------
SQRT_LN2_X2 = 1.6651092223153954    # 2 sqrt(ln 2) = sqrt(-2 ln(1/4))
SQRT_2LN2 = 1.1774100225154747      # sqrt(2 ln 2), sqrt(-2 ln(1/4)) cos(pi/4)


def _y_for_u1(u1_24bit):   # u1 = (y>>8 + 1) 2^-24
    return ((u1_24bit - 1) << 8) | 0xAB


def test_normal_special_cases():
    mu, sd = 0.5, 0.05
    # u1 = 1 -> ln u1 = 0 -> z = 0 exactly, whatever u2
    for y1 in (0, 123 << 8, 0xFFFFFFFF):
        assert oracle.normal_weight(0xFFFFFFFF, y1, mu, sd) == mu
    y0 = _y_for_u1(1 << 22)          # u1 = 1/4
    assert oracle.normal_weight(y0, 0, 0.0, 1.0) == pytest.approx(SQRT_LN2_X2, rel=1e-15)
    assert oracle.normal_weight(y0, 1 << 31, 0.0, 1.0) == pytest.approx(-SQRT_LN2_X2, rel=1e-15)  # u2 = 1/2
    assert abs(oracle.normal_weight(y0, 1 << 30, 0.0, 1.0)) < 1e-15                              # u2 = 1/4
    assert oracle.normal_weight(y0, 1 << 29, 0.0, 1.0) == pytest.approx(SQRT_2LN2, rel=1e-15)     # u2 = 1/8
    assert oracle.normal_weight(y0, 7 << 29, 0.0, 1.0) == pytest.approx(SQRT_2LN2, rel=1e-15)     # u2 = 7/8
    # the smallest u1 = 2^-24 gives the largest |z| = sqrt(48 ln 2)
    assert oracle.normal_weight(0x000000FF, 0, 0.0, 1.0) == pytest.approx(5.768107546403532068, rel=1e-14)
    # affine in (mu, sd)
    z = oracle.normal_weight(y0, 1 << 29, 0.0, 1.0)
    assert oracle.normal_weight(y0, 1 << 29, -0.5, 0.05) == pytest.approx(-0.5 + 0.05 * z, rel=1e-15)


def test_normal_sine_branch_special_cases():
    y0 = _y_for_u1(1 << 22)          # u1 = 1/4, radius 2 sqrt(ln 2)
    assert oracle.normal_weight(y0, 0, 0.0, 1.0, branch=1) == 0.0                                      # u2 = 0
    assert oracle.normal_weight(y0, 1 << 30, 0.0, 1.0, branch=1) == pytest.approx(SQRT_LN2_X2, rel=1e-15)   # 1/4
    assert oracle.normal_weight(y0, 3 << 30, 0.0, 1.0, branch=1) == pytest.approx(-SQRT_LN2_X2, rel=1e-15)  # 3/4
    assert oracle.normal_weight(y0, 1 << 29, 0.0, 1.0, branch=1) == pytest.approx(SQRT_2LN2, rel=1e-15)     # 1/8
    assert oracle.normal_weight(y0, 5 << 29, 0.0, 1.0, branch=1) == pytest.approx(-SQRT_2LN2, rel=1e-15)    # 5/8
    for y1 in (0, 123 << 8, 0xFFFFFFFF):
        assert oracle.normal_weight(0xFFFFFFFF, y1, 0.5, 0.05, branch=1) == 0.5


def test_normal_pair_radius():
    # both outputs of one pair lie on the circle of radius sqrt(-2 ln u1)
    for i in range(200):
        y0, y1 = oracle.word(3, 1, 1, 2 * i), oracle.word(3, 1, 1, 2 * i + 1)
        zc = oracle.normal_weight(y0, y1, 0.0, 1.0)
        zs = oracle.normal_weight(y0, y1, 0.0, 1.0, branch=1)
        u1 = ((y0 >> 8) + 1) * 2.0**-24
        assert zc * zc + zs * zs == pytest.approx(-2.0 * math.log(u1), rel=1e-12, abs=1e-300)


def test_normal_distribution():
    n = 100_000
    ws = np.array([oracle.normal_weight(oracle.word(7, 2, 1, 2 * i), oracle.word(7, 2, 1, 2 * i + 1),
                                        0.5, 0.05) for i in range(n)])
    assert stats.kstest(ws, "norm", args=(0.5, 0.05)).pvalue > 1e-4
    assert abs(ws.mean() - 0.5) < 4 * 0.05 / np.sqrt(n)
    wsin = np.array([oracle.normal_weight(oracle.word(7, 2, 1, 2 * i), oracle.word(7, 2, 1, 2 * i + 1),
                                          0.5, 0.05, branch=1) for i in range(n)])
    assert stats.kstest(wsin, "norm", args=(0.5, 0.05)).pvalue > 1e-4
    # the two outputs of a pair are independent: uncorrelated across pairs
    assert abs(np.corrcoef(ws, wsin)[0, 1]) < 4 / np.sqrt(n)
    # variance: (n-1) s^2 / sigma^2 ~ chi2(n-1)
    chi = (n - 1) * ws.var(ddof=1) / 0.05**2
    assert stats.chi2.sf(chi, n - 1) > 1e-4 and stats.chi2.cdf(chi, n - 1) > 1e-4


def test_uniform_weight():
    assert oracle.uniform_weight(0, -1.0, 3.0) == -1.0
    assert oracle.uniform_weight(0xFFFFFFFF, -1.0, 3.0) == 3.0 - 4.0 * 2.0**-24
    assert oracle.uniform_weight(1 << 31, -1.0, 3.0) == 1.0
    ws = np.array([oracle.uniform_weight(oracle.word(5, 0, 1, i), 2.0, 4.0) for i in range(50_000)])
    assert stats.kstest(ws, "uniform", args=(2.0, 2.0)).pvalue > 1e-4


def test_delay_steps_rounding():
    # exact quotients
    assert oracle.delay_steps(3.0, 1.0) == 3
    assert oracle.delay_steps(1.5, 0.5) == 3
    # ties go to even: 2.5 -> 2, 3.5 -> 4
    assert oracle.delay_steps(1.25, 0.5) == 2
    assert oracle.delay_steps(1.75, 0.5) == 4
    # below one step -> one step
    assert oracle.delay_steps(0.2, 0.5) == 1
    assert oracle.delay_steps(0.0, 0.1) == 1
    # fp32 evaluation: 0.3f / 0.1f rounds to 3 steps
    assert oracle.delay_steps(0.3, 0.1) == 3
    assert oracle.delay_steps(1.0, 0.1) == 10


def test_uniform_ms_delay():
    # x = 0 -> lo; delays in [lo, hi) ms with h = 0.5 -> steps in {rint(lo/h) .. rint(hi/h)}
    assert oracle.uniform_ms_delay(0, 1.0, 2.0, 0.5) == 2
    vals = [oracle.uniform_ms_delay(oracle.word(11, 0, 0, q), 1.0, 2.0, 0.5) for q in range(20000)]
    # d/h uniform on [2, 4): rint gives 2 on [2,2.5], 3 on (2.5,3.5), 4 on [3.5,4)
    cnt = np.bincount(vals, minlength=5)[2:5]
    expected = np.array([0.25, 0.5, 0.25]) * len(vals)
    assert stats.chisquare(cnt, expected).pvalue > 1e-4
