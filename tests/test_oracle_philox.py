"""Pins of the oracle's Philox4x32-10 and CountSketch hash against things other
than the oracle itself: published known answers, rocRAND's independent
Philox implementation (a header-only library, compiled here for the host),
exact big-integer arithmetic and distributional properties."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle.philox import philox4x32
from oracle.sketch import cs_hash, cs_hash_bigint


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = philox4x32(np.array(ctr), np.array(key))
        assert [int(v) for v in got] == out


_ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Eng : rocrand_device::philox4x32_10_engine {
  using philox4x32_10_engine::ten_rounds;
};
int main() {
  Eng e; unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def _rocrand_exe(tmp):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    gxx = shutil.which("g++")
    if not (os.path.exists(hdr) and gxx):
        pytest.skip("rocRAND headers or g++ not available")
    src = os.path.join(tmp, "p.cpp")
    exe = os.path.join(tmp, "p")
    with open(src, "w") as f:
        f.write(_ROCRAND_SRC)
    subprocess.run([gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    src, "-o", exe], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand_host():
    rng = np.random.default_rng(123)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64)
    ctr[:5] = [[0, 0, 0, 0], [2**32 - 1] * 4, [5, 0, 0, 0], [7, 1, 0, 0], [9, 0, 3, 1]]
    with tempfile.TemporaryDirectory() as tmp:
        exe = _rocrand_exe(tmp)
        inp = "\n".join(" ".join("%x" % int(v) for v in list(c) + list(k))
                        for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                             check=True).stdout.split()
    want = np.array([int(t, 16) for t in out], dtype=np.uint64).reshape(-1, 4)
    got = philox4x32(ctr, key)
    np.testing.assert_array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("r", [1, 2, 3, 6, 2500, 250000, 1000000, 2**31 + 11, 2**32 - 1])
def test_hash_range_reduction_exact(r):
    """The uint64 split form of floor(X*r/2^64) equals exact integer arithmetic."""
    seed = 0xDEADBEEF12345
    rows = [0, 1, 2, 12345, 2**31 - 1, 2**32 + 5, 9_999_999]
    for i in rows:
        h, s = cs_hash(1, r, seed, row0=i)
        hb, sb = cs_hash_bigint(i, r, seed)
        assert int(h[0]) == hb and int(s[0]) == sb
        assert 0 <= hb < r


def test_hash_uniform_and_signs_balanced():
    from scipy import stats
    n, r = 400_000, 97
    h, s = cs_hash(n, r, seed=2024)
    counts = np.bincount(h, minlength=r)
    chi2 = ((counts - n / r) ** 2 / (n / r)).sum()
    p = stats.chi2.sf(chi2, r - 1)
    assert p > 1e-4, (chi2, p)
    # sign balance: |mean| within 5 sigma of a fair coin
    assert abs(s.mean()) < 5.0 / np.sqrt(n)
    # hash and sign are not correlated
    assert abs(np.corrcoef(h, s)[0, 1]) < 5.0 / np.sqrt(n)


def test_hash_depends_on_seed_and_row_only():
    a, sa = cs_hash(1000, 4096, seed=5, row0=100)
    b, sb = cs_hash(2000, 4096, seed=5, row0=0)
    np.testing.assert_array_equal(a, b[100:1100])
    np.testing.assert_array_equal(sa, sb[100:1100])
    c, _ = cs_hash(1000, 4096, seed=6, row0=100)
    assert (a != c).mean() > 0.99
