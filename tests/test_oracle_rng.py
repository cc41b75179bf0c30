"""Pins of the oracle's random-number layer: Philox4x32-10 words, the uniform
map, Box-Muller, and the (path, step, block) counter layout."""
import math
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle

ROCRAND_CHECKER = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long blk = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_init(seed, sub, 0, &st);
    for (int i = 0; i < 4; ++i) skipahead(blk, &st);   /* 4 numbers per block */
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def _rocrand_words(cases):
    """Run rocRAND's own Philox4x32-10 (header library, host build) on
    (counter, key) cases; an external implementation, not ours."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers or hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "rr.cpp")
        exe = os.path.join(d, "rr")
        with open(src, "w") as f:
            f.write(ROCRAND_CHECKER)
        subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                       check=True, capture_output=True)
        inp = "\n".join(" ".join(str(x) for x in c + k) for c, k in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(x) for x in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand():
    rng = np.random.default_rng(123)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
             ([1, 2, 3, 4], [5, 6])]
    for _ in range(200):
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        k = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        cases.append((c, k))
    # the counters the pricing path uses: (p lo, step, block, p hi), key = seed
    for p, k, j, seed in [(0, 0, 0, 42), (1023, 63, 0, 42), (24999, 251, 2, 42),
                          (2**32 + 7, 5, 9, 2**40 + 3)]:
        cases.append(([p & 0xFFFFFFFF, k, j, p >> 32], [seed & 0xFFFFFFFF, seed >> 32]))
    ref = _rocrand_words(cases)
    ours = [oracle.philox(c, k) for c, k in cases]
    assert ours == ref


def test_uniform_map_exact():
    # exact rational value (2*(w>>9)+1) / 2^24 on edge and random words
    rng = np.random.default_rng(5)
    words = [0, 1, 511, 512, 513, 2**31, 2**32 - 1, 2**32 - 512]
    words += [int(x) for x in rng.integers(0, 2**32, 20000, dtype=np.uint64)]
    for w in words:
        u = oracle.uniform(w)
        assert Fraction(u) == Fraction(2 * (w >> 9) + 1, 2**24)
        assert 0.0 < u < 1.0
    assert oracle.uniform(0) == 2.0**-24
    assert oracle.uniform(2**32 - 1) == 1.0 - 2.0**-24


def test_uniform_values_exact_in_fp32():
    # all 2^23 values (2i+1) 2^-24 are exactly representable in FP32, so an
    # FP32 path and an FP64 path consume bit-identical uniforms
    i = np.arange(2**23, dtype=np.int64)
    v64 = (2 * i + 1).astype(np.float64) * 2.0**-24
    v32 = (2 * i + 1).astype(np.float32) * np.float32(2.0**-24)
    assert np.array_equal(v32.astype(np.float64), v64)


def test_box_muller_high_precision():
    mpmath.mp.prec = 120
    rng = np.random.default_rng(9)
    worst = 0.0
    pairs = [(0, 0), (2**32 - 1, 2**32 - 1), (0, 2**31), (2**31, 2**30)]
    pairs += [tuple(int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)) for _ in range(3000)]
    for w1, w2 in pairs:
        u1 = mpmath.mpf(2 * (w1 >> 9) + 1) / 2**24
        u2 = mpmath.mpf(2 * (w2 >> 9) + 1) / 2**24
        R = mpmath.sqrt(-2 * mpmath.log(u1))
        e_ref = float(R * mpmath.cos(2 * mpmath.pi * u2))
        h_ref = float(R * mpmath.sin(2 * mpmath.pi * u2))
        e, h = oracle.normal_pair(w1, w2)
        worst = max(worst, abs(e - e_ref), abs(h - h_ref))
    # a few ulp of |Z| <= 5.8
    assert worst < 4e-15


def test_normals_counter_layout():
    # asset 2j takes words (w0,w1) and asset 2j+1 words (w2,w3) of Philox
    # block j at counter (p lo, step, j, p hi) under key (seed lo, seed hi)
    for N, seed, p, k in [(1, 42, 0, 0), (5, 42, 1234, 17), (4, 7, 2**33 + 5, 250),
                          (20, 2**35 + 9, 99, 503)]:
        eps, eta = oracle.normals(N, seed, p, k)
        for a in range(N):
            j = a // 2
            w = oracle.philox([p & 0xFFFFFFFF, k, j, p >> 32], [seed & 0xFFFFFFFF, seed >> 32])
            pair = (w[0], w[1]) if a % 2 == 0 else (w[2], w[3])
            e, h = oracle.normal_pair(*pair)
            assert eps[a] == e and eta[a] == h


def test_normals_moments():
    # 2 x 400k Box-Muller draws: mean 0, variance 1, kurtosis 3, eps/eta uncorrelated
    N = 8
    eps = []
    eta = []
    for p in range(50000):
        e, h = oracle.normals(N, 42, p, 3)
        eps.append(e)
        eta.append(h)
    eps = np.concatenate(eps)
    eta = np.concatenate(eta)
    for z in (eps, eta):
        n = z.size
        assert abs(z.mean()) < 4.0 / math.sqrt(n)
        assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
        assert abs((z**4).mean() - 3.0) < 4.0 * math.sqrt(96.0 / n)
        assert np.abs(z).max() < 5.8
    assert abs(np.mean(eps * eta)) < 4.0 / math.sqrt(eps.size)
    # different assets of a path are uncorrelated
    E = eps.reshape(-1, N)
    c = np.corrcoef(E.T)
    assert np.abs(c - np.eye(N)).max() < 4.0 / math.sqrt(E.shape[0])
