"""The operand-validity predicates of the library (csrc/csr_check.hpp,
host-callable) compiled for the CPU and run over well-formed and malformed
CSR matrices and over values with NaN and infinities.  The expected codes
come from the CSR definition of the paper's Section 1 notation (offsets from
0 to nnz, never decreasing; column indices in [0, d)), cross-checked with
SciPy's own full format check on random cases."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# stdin: n d nnz, then n+1 offsets, nnz indices, nnz values (as doubles);
# prints the OR of every row, index and value code, and the same with the
# values narrowed to float
SRC = r"""
#include "paper_2203_02798_amd/csrc/csr_check.hpp"
#include <cstdio>
#include <vector>
int main() {
  long long n, d, nnz;
  while (scanf("%lld %lld %lld", &n, &d, &nnz) == 3) {
    std::vector<long long> ptr(n + 1);
    std::vector<long long> idx(nnz);
    std::vector<double> val(nnz);
    for (auto &p : ptr) scanf("%lld", &p);
    for (auto &c : idx) scanf("%lld", &c);
    for (auto &v : val) scanf("%lf", &v);
    unsigned code = 0, code32 = 0;
    for (long long i = 0; i < n; ++i) code |= psk::csr_row_code(ptr[i], ptr[i + 1], i, n, nnz);
    for (long long k = 0; k < nnz; ++k) code |= psk::csr_index_code((int)idx[k], d);
    code32 = code;
    for (long long k = 0; k < nnz; ++k) {
      code |= psk::value_code(val[k]);
      code32 |= psk::value_code((float)val[k]);
    }
    printf("%u %u\n", code, code32);
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
    src = os.path.join(tmp, "c.cpp")
    out = os.path.join(tmp, "c")
    with open(src, "w") as f:
        f.write(SRC)
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", ROOT, src,
                    "-o", out], check=True, capture_output=True)
    yield out
    shutil.rmtree(tmp, ignore_errors=True)


def run(exe, cases):
    lines = []
    for n, d, ptr, idx, val in cases:
        lines.append(f"{n} {d} {len(idx)}")
        lines.append(" ".join(str(int(p)) for p in ptr))
        lines.append(" ".join(str(int(c)) for c in idx))
        lines.append(" ".join(repr(float(v)) for v in val))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True)
    return [tuple(int(t) for t in ln.split()) for ln in res.stdout.splitlines()]


def good(n=5, d=7, seed=0):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, d + 1, n)
    ptr = np.concatenate([[0], np.cumsum(counts)])
    idx = np.concatenate([rng.permutation(d)[:c] for c in counts]).astype(np.int64)
    val = rng.standard_normal(len(idx))
    return n, d, ptr, idx, val


def test_named_cases(exe):
    """Each break of the definition alone, and the well-formed neighbours."""
    n, d, ptr, idx, val = good()
    nnz = len(idx)
    assert nnz > 3
    cases, want = [], []

    def add(p, i, v, code):
        cases.append((n, d, p, i, v))
        want.append(code)

    add(ptr, idx, val, 0)
    p = ptr.copy(); p[0] = 1                     # offsets must start at 0
    add(p, idx, val, 1)
    p = ptr.copy(); p[-1] = nnz - 1              # ... and end at nnz
    add(p, idx, val, 1)
    p = ptr.copy(); p[-1] = nnz + 1
    add(p, idx, val, 1)
    p = ptr.copy(); k = int(np.argmax(np.diff(ptr) > 0)) + 1
    p[k] = p[k + 1] + 1 if k + 1 <= n else p[k]  # one offset above its successor
    add(p, idx, val, 1)
    i2 = idx.copy(); i2[2] = d                   # index one past the last column
    add(ptr, i2, val, 1)
    i2 = idx.copy(); i2[1] = -1                  # negative index
    add(ptr, i2, val, 1)
    i2 = idx.copy(); i2[0] = d - 1               # the last column is fine
    add(ptr, i2, val, 0)
    for bad in (np.nan, np.inf, -np.inf):
        v2 = val.copy(); v2[3] = bad
        add(ptr, idx, v2, 2)
    i2 = idx.copy(); i2[0] = d
    v2 = val.copy(); v2[0] = np.nan
    add(ptr, i2, v2, 3)                          # both bits
    v2 = val.copy(); v2[0] = np.finfo(np.float64).max
    add(ptr, idx, v2, 0)                         # largest finite value
    # empty rows everywhere, and a matrix with no entries at all
    cases.append((3, 4, np.zeros(4, np.int64), np.zeros(0, np.int64), np.zeros(0)))
    want.append(0)
    cases.append((3, 4, np.array([0, 0, 0, 1]), np.zeros(0, np.int64), np.zeros(0)))
    want.append(1)
    got = run(exe, cases)
    assert [g[0] for g in got] == want


def test_float_narrowing(exe):
    """A double that overflows float is non-finite once narrowed: the FP32
    predicate sees the narrowed value."""
    n, d, ptr, idx, val = good(seed=3)
    v2 = val.copy(); v2[0] = 1e300
    got = run(exe, [(n, d, ptr, idx, v2)])
    assert got[0] == (0, 2)


def scipy_structure_ok(n, d, ptr, idx):
    if ptr[0] != 0 or ptr[-1] != len(idx):
        return False
    try:
        m = sp.csr_matrix((np.ones(len(idx)), idx.astype(np.int64), ptr.astype(np.int64)),
                          shape=(n, d))
        m.check_format(full_check=True)
    except ValueError:
        return False
    return True


def test_random_against_scipy(exe):
    """Random perturbations of well-formed matrices: the structure bit equals
    the negation of SciPy's full format check (plus its end offset)."""
    rng = np.random.default_rng(11)
    cases = []
    for t in range(300):
        n, d, ptr, idx, val = good(n=int(rng.integers(1, 9)), d=int(rng.integers(1, 9)),
                                   seed=100 + t)
        ptr, idx = ptr.copy(), idx.copy()
        what = rng.integers(0, 4)
        if what == 1 and len(ptr) > 1:
            j = rng.integers(0, len(ptr))
            ptr[j] += rng.integers(-2, 3)
        elif what == 2 and len(idx):
            idx[rng.integers(0, len(idx))] = rng.integers(-2, d + 3)
        cases.append((n, d, ptr, idx, val))
    got = run(exe, cases)
    for (n, d, ptr, idx, _), g in zip(cases, got):
        assert (g[0] & 1) == (0 if scipy_structure_ok(n, d, ptr, idx) else 1)
