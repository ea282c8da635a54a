"""Pins for the oracle's Philox generator and Gaussian test matrix.

What pins it (none of these re-types the oracle's own formulas):
* the same generic Philox code, instantiated at W = 64, reproduces numpy's
  independent Philox4x64-10 bit generator word for word (round function,
  key schedule, multiply-high/low and word permutation);
* the Weyl key increments equal the fractional parts of the golden ratio and
  of sqrt(3) in fixed point, computed here with exact integer square roots;
* the limb-wise multiply-high/low equals Python's exact big-integer product;
* the Box-Muller output is standard normal (moments, Kolmogorov-Smirnov),
  columns are uncorrelated, and the tail is bounded as 24-bit uniforms imply.
* the 32-bit instance that Omega uses reproduces the published Philox4x32
  known-answer vectors (tests/golden/philox4x32_kat.txt, 7 and 10 rounds);
* the raw Omega words (counter (g, j, stream, 0), key = seed) equal those of
  rocRAND's Philox4x32-10 engine, an independent implementation compiled
  from its header and run on the host, on 12 000 blocks.
"""

import os
import shutil
import subprocess
from math import isqrt, log, sqrt

import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("key,ctr", [((1, 2), (5, 0, 0, 0)),
                                     ((0, 0), (0, 0, 0, 0)),
                                     ((0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF),
                                      (0xFFFFFFFFFFFFFFF0, 7, 9, 0x8000000000000000))])
def test_generic_philox_w64_matches_numpy_philox(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    raw = bg.random_raw(12)
    # numpy advances its 256-bit counter before each block.
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    blocks = []
    for i in range(1, 4):
        ci = (c + i) % (1 << 256)
        blocks.append([(ci >> (64 * w)) & ((1 << 64) - 1) for w in range(4)])
    mine = philox.philox4(np.array(blocks, dtype=np.uint64), np.array(key, dtype=np.uint64), width=64)
    assert np.array_equal(mine.ravel(), raw)


@pytest.mark.parametrize("width", [32, 64])
def test_weyl_constants_are_golden_ratio_and_sqrt3(width):
    c = philox._CONSTANTS[width]
    golden_frac = (isqrt(5 << (2 * width)) - (1 << width)) // 2      # floor(2^W (phi - 1))
    sqrt3_frac = isqrt(3 << (2 * width)) - (1 << width)               # floor(2^W (sqrt 3 - 1))
    assert c["W0"] == golden_frac
    assert c["W1"] == sqrt3_frac


@pytest.mark.parametrize("width", [32, 64])
def test_mulhilo_against_big_integers(width):
    rng = np.random.default_rng(0)
    a = rng.integers(0, 1 << width, size=200, dtype=np.uint64, endpoint=False) if width < 64 else \
        rng.integers(0, 2 ** 63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = np.uint64(philox._CONSTANTS[width]["M0"])
    hi, lo = philox.mulhilo(b, a, width)
    for x, h, lw in zip(a, hi, lo):
        prod = int(b) * int(x)
        assert int(h) == prod >> width
        assert int(lw) == prod & ((1 << width) - 1)


def test_omega_is_standard_normal():
    Om = philox.omega(seed=0, n=20000, l=50)
    z = Om.ravel()
    assert abs(z.mean()) < 5.0 / sqrt(z.size)
    assert abs(z.var() - 1.0) < 6.0 * sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # excess kurtosis and skewness of a normal are 0
    assert abs(stats.skew(z)) < 0.02 and abs(stats.kurtosis(z)) < 0.04
    # both Box-Muller branches (even and odd rows) and both word pairs are normal
    for r in range(4):
        assert stats.kstest(Om[r::4].ravel(), "norm").pvalue > 1e-4
    C = np.corrcoef(Om.T)
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert np.max(np.abs(off)) < 6.0 / sqrt(Om.shape[0])
    # the two rows of a Box-Muller pair, and the two pairs of a block, are independent
    for a, b in [(0, 1), (2, 3), (0, 2), (1, 3)]:
        r = np.corrcoef(Om[a::4].ravel(), Om[b::4].ravel())[0, 1]
        assert abs(r) < 6.0 / sqrt(Om[a::4].size)


def test_omega_tail_bound_and_exact_uniforms():
    # u1 >= 2^-24, so |z| <= sqrt(-2 ln 2^-24)
    Om = philox.omega(seed=123, n=4096, l=64)
    assert np.max(np.abs(Om)) <= sqrt(2.0 * 24.0 * log(2.0)) + 1e-12
    u1, u2 = philox.uniform_pair(np.array([0, 0xFFFFFFFF], dtype=np.uint64),
                                 np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert u1[0] == 2.0 ** -24 and u1[1] == 1.0
    assert u2[0] == 0.0 and u2[1] == 1.0 - 2.0 ** -24
    # the uniforms are exact in float32
    assert np.all(u1.astype(np.float32).astype(np.float64) == u1)


def test_omega_layout_prefix_seed_and_stream():
    a = philox.omega(seed=7, n=37, l=9)
    b = philox.omega(seed=7, n=37, l=20)
    assert np.array_equal(a, b[:, :9])              # narrower Omega is a prefix
    c = philox.omega(seed=7, n=41, l=9)
    assert np.array_equal(a, c[:37])                # row i does not depend on n
    assert not np.allclose(a, philox.omega(seed=8, n=37, l=9))
    assert not np.allclose(a, philox.omega(seed=7, n=37, l=9, stream=1))
    # key uses both halves of a 64-bit seed
    assert not np.allclose(philox.omega(seed=1, n=8, l=2), philox.omega(seed=1 + (1 << 32), n=8, l=2))
    # element (i, j) comes from block (i // 4, j): four rows per block
    w = philox.philox_words(7, np.array([[2, 3]]))[0]
    u1, u2 = philox.uniform_pair(w[2], w[3])
    r = sqrt(-2.0 * log(float(u1)))
    assert a[10, 3] == pytest.approx(r * np.cos(2 * np.pi * float(u2)), rel=1e-15, abs=1e-15)
    assert a[11, 3] == pytest.approx(r * np.sin(2 * np.pi * float(u2)), rel=1e-15, abs=1e-15)


def test_omega_empty():
    assert philox.omega(0, 0, 5).shape == (0, 5)
    assert philox.omega(0, 5, 0).shape == (5, 0)


HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows.append((int(t[0]), [int(x, 16) for x in t[1:5]], [int(x, 16) for x in t[5:7]],
                             [int(x, 16) for x in t[7:11]]))
    return rows


@pytest.mark.parametrize("rounds,ctr,key,expect", _kat_rows())
def test_philox4x32_known_answers(rounds, ctr, key, expect):
    got = philox.philox4(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64), width=32, rounds=rounds)
    assert [int(x) for x in got] == expect


def _build_rocrand_words(tmp_path):
    src = os.path.join(HERE, "rocrand_philox_words.cpp")
    exe = str(tmp_path / "rocrand_philox_words")
    inc = "/opt/rocm/include"
    if not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers not installed")
    for cxx in (shutil.which("g++"), "/opt/rocm/bin/hipcc"):
        if cxx and os.path.exists(cxx):
            r = subprocess.run([cxx, "-O2", "-x", "c++", "-I", inc, "-D__HIP_PLATFORM_AMD__", src, "-o", exe],
                               capture_output=True, text=True)
            if r.returncode == 0:
                return exe
    pytest.skip("no host compiler could build the rocRAND helper")


def test_omega_words_match_rocrand_engine(tmp_path):
    exe = _build_rocrand_words(tmp_path)
    rng = np.random.default_rng(11)
    lines, cases = [], []
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        for stream in (0, 1, 2):
            ctr = np.concatenate([rng.integers(0, 2 ** 32, size=(1330, 2), dtype=np.uint64),
                                  np.array([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [1, 0], [0, 1]], dtype=np.uint64)])
            cases.append((seed, stream, ctr))
            lines += [f"{seed} {stream} {int(g)} {int(j)}" for g, j in ctr]
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    ref = np.array([[int(x, 16) for x in ln.split()] for ln in r.stdout.splitlines()], dtype=np.uint64)
    assert ref.shape == (len(lines), 4) and len(lines) >= 12000
    mine = np.concatenate([philox.philox_words(seed, ctr, stream) for seed, stream, ctr in cases]).astype(np.uint64)
    assert np.array_equal(mine, ref)
