"""The library's random-number and Box-Muller arithmetic (csrc/common.hpp,
host-callable) compiled for the CPU and checked against the oracle and
NumPy: Philox and the CountSketch hash bit for bit, the lean log and
sin/cos(pi z) to about one ulp, the normals to 1e-14."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import sketch as osk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r"""
#include "paper_2203_02798_amd/csrc/common.hpp"
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv) {
  const char *mode = argv[1];
  if (mode[0] == 'l') {            // log of doubles from stdin
    double x;
    while (scanf("%lf", &x) == 1) printf("%.17g\n", psk::bm_log(x));
  } else if (mode[0] == 's') {     // sin/cos(pi z)
    double z, s, c;
    while (scanf("%lf", &z) == 1) { psk::bm_sincospi(z, s, c); printf("%.17g %.17g\n", s, c); }
  } else if (mode[0] == 'g') {     // normals: q a seed
    unsigned long long q, seed; unsigned a;
    while (scanf("%llu %u %llu", &q, &a, &seed) == 3) {
      double z[4]; psk::gauss4_f64(q, a, seed, z);
      printf("%.17g %.17g %.17g %.17g\n", z[0], z[1], z[2], z[3]);
    }
  } else if (mode[0] == 'h') {     // hash: i r seed
    unsigned long long i, seed; unsigned r;
    while (scanf("%llu %u %llu", &i, &r, &seed) == 3) {
      unsigned h, neg; psk::cs_hash_row(i, r, seed, h, neg);
      printf("%u %u\n", h, neg);
    }
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def exe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    tmp = tempfile.mkdtemp()
    src = os.path.join(tmp, "m.cpp")
    out = os.path.join(tmp, "m")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", ROOT,
                    "-I", os.path.join(ROOT, "include"), src, "-o", out],
                   check=True, capture_output=True)
    yield out
    shutil.rmtree(tmp, ignore_errors=True)


def _run(exe, mode, lines):
    p = subprocess.run([exe, mode], input="\n".join(lines), capture_output=True,
                       text=True, check=True)
    return np.array([[float(t) for t in l.split()] for l in p.stdout.splitlines()])


def test_bm_log(exe):
    rng = np.random.default_rng(0)
    x = np.concatenate([(rng.integers(0, 2**32, 20000) + 0.5) * 2.0 ** -32,
                        [2.0 ** -33, 0.5, 1.0 - 2.0 ** -33, 0.70710678118654752,
                         0.7071067811865476, 1e-300, 1.0]])
    got = _run(exe, "l", [repr(float(v)) for v in x])[:, 0]
    ref = np.log(x)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    assert err.max() < 4e-16, (err.max(), x[err.argmax()])


def test_bm_sincospi(exe):
    rng = np.random.default_rng(1)
    z = np.concatenate([2.0 * (rng.integers(0, 2**32, 20000) + 0.5) * 2.0 ** -32,
                        [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 0.125, 1e-9]])
    got = _run(exe, "s", [repr(float(v)) for v in z])
    # reference by the exact reduction z - k/2 in FP64 then libm of pi*y
    k = np.rint(2 * z)
    y = z - k / 2
    q = k.astype(np.int64) & 3
    sp, cp = np.sin(np.pi * y), np.cos(np.pi * y)
    sref = np.choose(q, [sp, cp, -sp, -cp])
    cref = np.choose(q, [cp, -sp, -cp, sp])
    assert np.abs(got[:, 0] - sref).max() < 4e-16
    assert np.abs(got[:, 1] - cref).max() < 4e-16
    # and against sin/cos(2 pi u) as the oracle evaluates them
    np.testing.assert_allclose(got[:, 0], np.sin(np.pi * z), rtol=0, atol=2e-15)
    np.testing.assert_allclose(got[:, 1], np.cos(np.pi * z), rtol=0, atol=2e-15)


def test_gauss4_matches_oracle(exe):
    rng = np.random.default_rng(2)
    rows = []
    for t in range(300):
        q = int(rng.integers(0, 2**40)) if t % 3 else t
        a = int(rng.integers(0, 5000))
        seed = int(rng.integers(0, 2**63))
        rows.append((q, a, seed))
    got = _run(exe, "g", [f"{q} {a} {s}" for q, a, s in rows])
    for (q, a, s), g in zip(rows, got):
        ref = osk.gaussian_normals(a + 1, 4 * q, 4 * q + 4, s)[a]
        np.testing.assert_allclose(g, ref, rtol=1e-14, atol=1e-14)


def test_hash_row_matches_oracle(exe):
    rng = np.random.default_rng(3)
    rows = [(int(rng.integers(0, 2**40)), int(rng.integers(1, 2**31)),
             int(rng.integers(0, 2**64, dtype=np.uint64))) for _ in range(500)]
    got = _run(exe, "h", [f"{i} {r} {s}" for i, r, s in rows])
    for (i, r, s), g in zip(rows, got):
        h, sg = osk.cs_hash(1, r, s, row0=i)
        assert int(g[0]) == int(h[0]) and (1 if sg[0] < 0 else 0) == int(g[1])
