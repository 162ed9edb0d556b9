"""Device path vs the FP64 oracle, element by element, on seeded inputs that
span several tiles with ragged tails.  Every call goes through the C ABI of
libpsk.so (via the ctypes binding)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from helpers import U32, U64, gamma, rel_fro, sketch_abs_bound, to_device
from oracle import gram as og
from oracle import css as ocss
from oracle import leverage as olev
from oracle import lsq as olsq
from oracle import sketch as osk

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_2203_02798_amd import api as a
    return a


def _say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# hash
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("row0,count,r,seed", [
    (0, 20000, 2500, 0), (0, 100000, 250000, 1), (123456789, 50000, 1_000_000, 7),
    (0, 4096, 1, 3), (2 ** 31 - 4096, 4096, 2 ** 31 - 1, 0xFFFFFFFFFFFFFFFF),
    (5, 0, 10, 2), (0, 777, 3, 0xDEADBEEF)])
def test_cs_hash_bit_exact(api, row0, count, r, seed):
    _say(f"cs_hash row0={row0} count={count} r={r}")
    h, s = api.cs_hash(count, r, seed, row0=row0)
    ho, so = osk.cs_hash(count, r, seed, row0=row0)
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.int64), ho)
    np.testing.assert_array_equal(s.cpu().numpy(), so)


# ---------------------------------------------------------------------------
# S*A
# ---------------------------------------------------------------------------
DENSE_CASES = [  # n, d, r
    (20000, 50, 2500), (3001, 37, 97), (4000, 257, 64), (5000, 512, 5000),
    (20000, 8, 4), (1000, 1, 2000), (777, 130, 1)]


@pytest.mark.parametrize("n,d,r", DENSE_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sketch_cs_dense_integer_bit_exact(api, n, d, r, dt):
    _say(f"sketch_cs dense int n={n} d={d} r={r} {dt}")
    npdt = np.float64 if dt == "f64" else np.float32
    a = synth.dense_integer(n, d, seed=n + d, lo=-4, hi=4, dtype=npdt)
    sa = api.sketch_cs(to_device(a), r, seed=11).cpu().numpy()
    np.testing.assert_array_equal(sa.astype(np.float64), osk.sketch_cs(a, r, 11))


@pytest.mark.parametrize("n,d,r", [(20000, 50, 2500), (3001, 37, 97), (4000, 257, 64),
                                   (20000, 8, 4), (777, 130, 1)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sketch_cs_dense_real_within_bound(api, n, d, r, dt):
    _say(f"sketch_cs dense real n={n} d={d} r={r} {dt}")
    npdt = np.float64 if dt == "f64" else np.float32
    a = synth.dense_gaussian(n, d, seed=3, dtype=npdt)
    sa = api.sketch_cs(to_device(a), r, seed=5).cpu().numpy().astype(np.float64)
    ref = osk.sketch_cs(a, r, 5)
    bound = sketch_abs_bound(a, r, 5, U64 if dt == "f64" else U32)
    assert np.all(np.abs(sa - ref) <= bound + 1e-300)


@pytest.mark.parametrize("kind,dt", [("dense", "f64"), ("csr", "f64"), ("dense", "f32"),
                                     ("csr", "f32")])
def test_sketch_cs_real_bit_exact_in_bin_order(api, kind, dt):
    """With r >= 8192 every bucket is summed by one wavefront, in increasing
    row order, in FP64: the oracle's S @ A (SciPy's CSR product, which adds
    the rows of each bucket in that same order) gives the same bits for real
    data too, which pins the binning order (FP32: one rounding of that same
    FP64 sum)."""
    npdt = np.float64 if dt == "f64" else np.float32
    a = (synth.dense_gaussian(200000, 40, seed=4, dtype=npdt) if kind == "dense"
         else synth.csr_uniform(300000, 70, 0.02, seed=4, dtype=npdt))
    r = 16384
    sa = api.sketch_cs(to_device(a), r, seed=9).cpu().numpy()
    ref = osk.sketch_cs(a, r, 9)
    if dt == "f32":
        ref = ref.astype(np.float32)
    np.testing.assert_array_equal(sa, ref)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_sketch_cs_f32_one_rounding(api, kind):
    """FP32 A: each bucket is summed in FP64 and rounded once to FP32, so
    |SA^ - SA| <= u32 |SA| + (1 + u32) gamma_k(u64) (|S||A|) componentwise
    (the FP32-sum bound gamma_k(u32) (|S||A|) is far looser)."""
    a = (synth.dense_gaussian(20000, 50, seed=3, dtype=np.float32) if kind == "dense"
         else synth.csr_uniform(50000, 64, 0.05, seed=3, dtype=np.float32))
    r = 512
    sa = api.sketch_cs(to_device(a), r, seed=5).cpu().numpy().astype(np.float64)
    ref = osk.sketch_cs(a, r, 5)
    bound = U32 * np.abs(ref) + (1 + U32) * sketch_abs_bound(a, r, 5, U64)
    assert np.all(np.abs(sa - ref) <= bound + 1e-300)


def test_sketch_cs_strided_rows(api):
    a = synth.dense_integer(3000, 64, seed=2)
    full = to_device(a)
    view = full[:, :50]  # ld = 64 > d = 50
    sa = api.sketch_cs(view, 301, seed=4).cpu().numpy()
    np.testing.assert_array_equal(sa, osk.sketch_cs(a[:, :50], 301, 4))


CSR_CASES = [  # n, d, density, r
    (20000, 500, 1e-3, 2500), (50000, 64, 0.05, 4096), (3000, 33, 0.2, 7),
    (1000, 700, 0.01, 100000), (4000, 16, 0.5, 1)]


@pytest.mark.parametrize("n,d,dens,r", CSR_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sketch_cs_csr_integer_bit_exact(api, n, d, dens, r, dt):
    _say(f"sketch_cs csr int n={n} d={d} r={r} {dt}")
    a = synth.csr_integer(n, d, dens, seed=9, dtype=np.float64)
    if dt == "f32":
        a = a.astype(np.float32)
    sa = api.sketch_cs(to_device(a), r, seed=13).cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(sa, osk.sketch_cs(a, r, 13))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sketch_cs_csr_zipf_real_within_bound(api, dt):
    npdt = np.float64 if dt == "f64" else np.float32
    a = synth.csr_zipf(100000, 300, 2e-3, seed=4, dtype=npdt)
    r = 20000
    sa = api.sketch_cs(to_device(a), r, seed=6).cpu().numpy().astype(np.float64)
    ref = osk.sketch_cs(a, r, 6)
    # CSR accumulation: per output entry at most (bucket rows) additions
    bound = sketch_abs_bound(a, r, 6, U64 if dt == "f64" else U32)
    assert np.all(np.abs(sa - ref) <= bound + 1e-300)


def test_sketch_cs_csr_empty_rows_and_empty_matrix(api):
    a = synth.csr_from_parts(1000, 20, [3, 3, 999], [1, 5, 19], [1.0, -2.0, 4.0])
    sa = api.sketch_cs(to_device(a), 50, seed=1).cpu().numpy()
    np.testing.assert_array_equal(sa, osk.sketch_cs(a, 50, 1))
    z = synth.csr_from_parts(500, 10, [], [], [])
    sa = api.sketch_cs(to_device(z), 40, seed=1).cpu().numpy()
    assert np.all(sa == 0)


@pytest.mark.parametrize("prec", ["f64", "bf16", "fp8"])
def test_csr_mostly_empty_rows(api, prec):
    """CSR A is binned over the rows that hold an entry only: a Zipf matrix
    with a few percent of its rows occupied gives the oracle's G*S*A in every
    precision and OSNAP S*A (s = 4) in bin order bit for bit on integers;
    an all-empty matrix and one whose only entries sit in its first and last
    rows give zero and the oracle's values."""
    from oracle import osnap as oo
    tol = {"f64": 1e-13, "bf16": 1e-4, "fp8": 1e-4}[prec]
    ref_gcs = {"f64": lambda a, m, r, s: osk.sketch_gcs(a, m, r, s),
               "bf16": osk.sketch_gcs_bf16_reference,
               "fp8": osk.sketch_gcs_fp8_reference}[prec]
    a = synth.csr_zipf(400_000, 120, 1e-3, seed=11, dtype=np.float32)
    occupied = int((np.diff(a.indptr) > 0).sum())
    _say(f"mostly empty {prec}: n={a.shape[0]} occupied={occupied} nnz={a.nnz}")
    assert occupied < a.shape[0] // 20
    A = to_device(a)
    for m, r in ((96, 4096), (33, 50000)):
        c = api.sketch_gcs(A, m, r, seed=8, prec=prec).cpu().numpy()
        e = rel_fro(c, ref_gcs(a, m, r, 8))
        _say(f"  G S A m={m} r={r}: {e:.3e}")
        assert e <= tol
    small = synth.csr_integer(2000, 30, 0.1, seed=3)
    srow = np.repeat(np.arange(2000), np.diff(small.indptr))
    place = np.sort(np.random.default_rng(3).choice(200_000, 2000, replace=False))
    ai = synth.csr_from_parts(200_000, 30, place[srow], small.indices, small.data)
    for s, r in ((4, 1024), (1, 777)):
        got = api.sketch_osnap(to_device(ai), s, 0, r, seed=5).cpu().numpy()
        np.testing.assert_array_equal(got, oo.sketch_osnap(ai, r, s, 5))
    z = synth.csr_from_parts(70_000, 12, [], [], [])
    assert np.all(api.sketch_osnap(to_device(z), 4, 0, 256, seed=1).cpu().numpy() == 0)
    assert np.all(api.sketch_osnap(to_device(z), 4, 16, 256, seed=1, prec=prec).cpu().numpy()
                  == 0)
    ends = synth.csr_from_parts(70_000, 12, [0, 0, 69_999], [2, 11, 5], [1.0, -3.0, 2.0])
    np.testing.assert_array_equal(api.sketch_osnap(to_device(ends), 2, 0, 64, seed=4).cpu().numpy(),
                                  oo.sketch_osnap(ends, 64, 2, 4))
    c = api.sketch_gcs(to_device(ends), 9, 64, seed=4, prec=prec).cpu().numpy()
    assert rel_fro(c, ref_gcs(ends, 9, 64, 4)) <= tol


# ---------------------------------------------------------------------------
# G*S*A (FP64)
# ---------------------------------------------------------------------------
def _gcs_input(kind, n, d):
    """'csr' (density 1e-3) or 'csr:<density>', 'dense32', 'dense'."""
    if kind.startswith("csr"):
        dens = float(kind.split(":")[1]) if ":" in kind else 1e-3
        return synth.csr_uniform(n, d, dens, seed=1)
    if kind == "dense32":
        return synth.dense_gaussian(n, d, seed=1, dtype=np.float32)
    if kind == "csr32":
        return synth.csr_uniform(n, d, 1e-3, seed=1, dtype=np.float32)
    return synth.dense_gaussian(n, d, seed=1)


@pytest.mark.parametrize("kind,n,d,m,r", [
    ("dense", 20000, 50, 200, 2500),      # the small dense FP64 workload
    ("dense", 6000, 130, 77, 3001),
    ("csr", 100000, 500, 300, 25000),
    # S*A sparse, d > 512 (16-row tiles), G blocks of about 6000 entries
    # (staged in several turns), ragged m
    ("csr", 50000, 1000, 77, 4096),
    ("dense32", 8000, 96, 129, 1024),
    ("csr32", 100000, 500, 300, 25000)])   # FP32 CSR through the sparse product
def test_sketch_gcs_f64(api, kind, n, d, m, r):
    _say(f"sketch_gcs {kind} n={n} d={d} m={m} r={r}")
    a = _gcs_input(kind, n, d)
    c = api.sketch_gcs(to_device(a), m, r, seed=21).cpu().numpy()
    ref = osk.sketch_gcs(a, m, r, 21)
    err = rel_fro(c, ref)
    _say(f"  rel err {err:.3e}")
    # FP32 A too: its entries are exact in FP64 and S*A is summed in FP64
    assert err <= 1e-12


def test_sketch_gcs_m0_is_sketch_cs(api):
    a = synth.dense_gaussian(3000, 20, seed=2)
    x = api.sketch_gcs(to_device(a), 0, 300, seed=3).cpu().numpy()
    y = api.sketch_cs(to_device(a), 300, seed=3).cpu().numpy()
    np.testing.assert_array_equal(x, y)


def test_sketch_gcs_deterministic(api):
    a = to_device(synth.csr_uniform(50000, 200, 5e-3, seed=3))
    c1 = api.sketch_gcs(a, 150, 8000, seed=5)
    c2 = api.sketch_gcs(a, 150, 8000, seed=5)
    assert torch.equal(c1, c2)


# ---------------------------------------------------------------------------
# G*S*A with bfloat16 operands (FP32 accumulation, FP64 split-K reduction)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,n,d,m,r", [
    ("dense", 20000, 50, 200, 2500),
    ("dense", 6000, 130, 77, 3001),
    ("dense", 3000, 600, 150, 1000),     # two 512-column tiles, ragged
    ("dense", 500, 3, 5, 7),             # one partial 32-bucket chunk
    ("csr", 100000, 500, 300, 25000),
    ("csr", 50000, 1000, 77, 4096),
    ("dense32", 8000, 96, 129, 1024)])
def test_sketch_gcs_bf16(api, kind, n, d, m, r):
    _say(f"sketch_gcs bf16 {kind} n={n} d={d} m={m} r={r}")
    a = _gcs_input(kind, n, d)
    c = api.sketch_gcs(to_device(a), m, r, seed=21, prec="bf16").cpu().numpy()
    # kernel arithmetic: against the exact product of the rounded operands
    e_arith = rel_fro(c, osk.sketch_gcs_bf16_reference(a, m, r, 21))
    # format loss: against the FP64 sketch
    e_fmt = rel_fro(c, osk.sketch_gcs(a, m, r, 21))
    _say(f"  vs quantised reference {e_arith:.3e}, vs FP64 {e_fmt:.3e}")
    assert e_arith <= 1e-4
    assert e_fmt <= 1e-2


# FP8 e4m3 with per-128-bucket power-of-two scales.  Kernel arithmetic is
# checked against the quantisation-aware product at 1e-4 normwise (the bar
# of the reduced-precision products): the device draws the normals in FP32,
# so about 2 in 1e6 of them round to the neighbouring e4m3 value of the FP64
# oracle's (relative quantum 2^-3), each moving C by about 0.1 / sqrt(m r)
# of its norm, and the FP32 accumulation adds ~1e-6.
@pytest.mark.parametrize("kind,n,d,m,r", [
    ("dense", 20000, 50, 200, 2500),
    ("dense", 6000, 130, 77, 3001),
    ("dense", 3000, 600, 150, 1000),     # two 512-column tiles, ragged
    ("dense", 500, 3, 5, 7),             # one partial 128-bucket chunk
    ("csr", 100000, 500, 300, 25000),
    # A with fewer than r d / 512 nonzeros: the product over the nonzeros
    # of S*A (512- and 1024-column forms)
    ("csr", 30000, 200, 100, 32768),
    ("csr:2e-4", 20000, 700, 77, 8192),
    ("dense32", 8000, 96, 129, 1024)])
def test_sketch_gcs_fp8(api, kind, n, d, m, r):
    _say(f"sketch_gcs fp8 {kind} n={n} d={d} m={m} r={r}")
    a = _gcs_input(kind, n, d)
    c = api.sketch_gcs(to_device(a), m, r, seed=21, prec="fp8").cpu().numpy()
    e_arith = rel_fro(c, osk.sketch_gcs_fp8_reference(a, m, r, 21))
    e_fmt = rel_fro(c, osk.sketch_gcs(a, m, r, 21))
    _say(f"  vs quantised reference {e_arith:.3e}, vs FP64 {e_fmt:.3e}")
    assert e_arith <= 1e-4
    assert e_fmt <= 1e-1


def test_sketch_gcs_fp8_deterministic(api):
    a = to_device(synth.csr_uniform(50000, 200, 5e-3, seed=3))
    c1 = api.sketch_gcs(a, 150, 8000, seed=5, prec="fp8")
    c2 = api.sketch_gcs(a, 150, 8000, seed=5, prec="fp8")
    assert torch.equal(c1, c2)


# ---------------------------------------------------------------------------
# G*A (Gaussian-only sketch, csrjlt)
# ---------------------------------------------------------------------------
def _g_input(kind, n, d):
    """'dense', 'dense32', 'dense_ld' (row stride > d), 'csr[:density]',
    'csr32' (FP32 values)."""
    if kind == "dense_ld":
        full = synth.dense_gaussian(n, d + 11, seed=2)
        return full[:, :d], torch.from_numpy(full).cuda()[:, :d]
    if kind == "csr32":
        a = synth.csr_uniform(n, d, 2e-3, seed=2, dtype=np.float32)
        return a, to_device(a)
    a = _gcs_input(kind, n, d)
    return a, to_device(a)


@pytest.mark.parametrize("kind,n,d,m", [
    ("dense", 20000, 50, 200),
    ("dense_ld", 5000, 37, 77),
    ("dense32", 8000, 96, 129),
    ("csr", 100000, 500, 300),
    ("csr:2e-2", 20000, 700, 77),        # d > 512; rows of ~14 entries
    ("csr32", 50000, 200, 100)])
def test_sketch_g_f64(api, kind, n, d, m):
    _say(f"sketch_g f64 {kind} n={n} d={d} m={m}")
    a, ad = _g_input(kind, n, d)
    c = api.sketch_g(ad, m, seed=13).cpu().numpy()
    err = rel_fro(c, osk.sketch_g(a, m, 13))
    _say(f"  rel err {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("prec,tol_arith,tol_fmt", [("bf16", 1e-4, 1e-2), ("fp8", 1e-4, 1e-1)])
@pytest.mark.parametrize("kind,n,d,m", [
    ("dense", 20000, 50, 200),
    ("csr", 40000, 300, 150),
    ("csr:2e-2", 20000, 700, 77)])
def test_sketch_g_reduced(api, prec, tol_arith, tol_fmt, kind, n, d, m):
    _say(f"sketch_g {prec} {kind} n={n} d={d} m={m}")
    a, ad = _g_input(kind, n, d)
    c = api.sketch_g(ad, m, seed=13, prec=prec).cpu().numpy()
    ref = (osk.sketch_g_bf16_reference if prec == "bf16" else osk.sketch_g_fp8_reference)
    e_arith = rel_fro(c, ref(a, m, 13))
    e_fmt = rel_fro(c, osk.sketch_g(a, m, 13))
    _say(f"  vs quantised reference {e_arith:.3e}, vs FP64 {e_fmt:.3e}")
    assert e_arith <= tol_arith
    assert e_fmt <= tol_fmt


@pytest.mark.parametrize("prec", ["f64", "bf16", "fp8"])
def test_sparse_products_degenerate_inputs(api, prec):
    """The products over the nonzeros (sketch_gcs of sparse S*A, sketch_g of
    CSR A) on empty and near-empty matrices and one-row G: an empty matrix
    gives exactly zero; one or three entries, m = 1 and n = 1 match the
    oracle (FP8/BF16 against their quantised references)."""
    tol = {"f64": 1e-13, "bf16": 1e-4, "fp8": 1e-4}[prec]
    ref_g = {"f64": lambda a, m, s: osk.sketch_g(a, m, s),
             "bf16": osk.sketch_g_bf16_reference, "fp8": osk.sketch_g_fp8_reference}[prec]
    ref_gcs = {"f64": lambda a, m, r, s: osk.sketch_gcs(a, m, r, s),
               "bf16": osk.sketch_gcs_bf16_reference,
               "fp8": osk.sketch_gcs_fp8_reference}[prec]
    z = synth.csr_from_parts(3000, 40, [], [], [])
    assert np.all(api.sketch_g(to_device(z), 7, seed=2, prec=prec).cpu().numpy() == 0)
    assert np.all(api.sketch_gcs(to_device(z), 7, 4096, seed=2, prec=prec).cpu().numpy() == 0)
    cases = [
        (synth.csr_from_parts(3000, 40, [1234], [17], [2.5]), 9, 4096),
        (synth.csr_from_parts(3000, 40, [0, 1234, 2999], [0, 17, 39], [1.0, -3.0, 0.5]), 1, 8192),
        (synth.csr_from_parts(1, 40, [0, 0], [3, 30], [1.5, -2.0]), 5, 1)]
    for a, m, r in cases:
        _say(f"degenerate {prec}: nnz={a.nnz} n={a.shape[0]} m={m} r={r}")
        c = api.sketch_g(to_device(a), m, seed=2, prec=prec).cpu().numpy()
        ref = ref_g(a, m, 2)
        assert rel_fro(c, ref) <= tol, ("sketch_g", rel_fro(c, ref))
        c = api.sketch_gcs(to_device(a), m, r, seed=2, prec=prec).cpu().numpy()
        ref = ref_gcs(a, m, r, 2)
        assert rel_fro(c, ref) <= tol, ("sketch_gcs", rel_fro(c, ref))


@pytest.mark.parametrize("prec", ["f64", "bf16", "fp8"])
def test_sparse_products_dense_column(api, prec):
    """A CSR matrix with one full column (an intercept, or b appended to A):
    in the products over the nonzeros that column fills whole G blocks and
    is summed by all threads of the workgroup together."""
    n, d, r, m = 100000, 500, 8192, 160
    a = synth.csr_uniform(n, d, 1e-4, seed=6).tolil()
    a[:, 7] = 1.0 + 0.001 * np.arange(n)[:, None]
    a = a.tocsr()
    tol = {"f64": 1e-12, "bf16": 1e-4, "fp8": 1e-4}[prec]
    ref_g = {"f64": lambda: osk.sketch_g(a, m, 3), "bf16": lambda: osk.sketch_g_bf16_reference(a, m, 3),
             "fp8": lambda: osk.sketch_g_fp8_reference(a, m, 3)}[prec]
    ref_gcs = {"f64": lambda: osk.sketch_gcs(a, m, r, 3),
               "bf16": lambda: osk.sketch_gcs_bf16_reference(a, m, r, 3),
               "fp8": lambda: osk.sketch_gcs_fp8_reference(a, m, r, 3)}[prec]
    ad = to_device(a)
    e1 = rel_fro(api.sketch_g(ad, m, seed=3, prec=prec).cpu().numpy(), ref_g())
    e2 = rel_fro(api.sketch_gcs(ad, m, r, seed=3, prec=prec).cpu().numpy(), ref_gcs())
    _say(f"dense column {prec}: sketch_g {e1:.3e}, sketch_gcs {e2:.3e}")
    assert e1 <= tol and e2 <= tol


def test_sketch_g_deterministic(api):
    a = to_device(synth.csr_uniform(50000, 200, 5e-3, seed=3))
    for prec in ("f64", "bf16", "fp8"):
        c1 = api.sketch_g(a, 150, seed=5, prec=prec)
        c2 = api.sketch_g(a, 150, seed=5, prec=prec)
        assert torch.equal(c1, c2), prec


@pytest.mark.parametrize("kind,cond,want", [("dense", 1.0, "fp8"), ("dense", 1e3, "f64"),
                                            ("csr", 1.0, "fp8"), ("csr", 1e3, "f64")])
def test_lsq_solve_fp8_sketch(api, kind, cond, want):
    # CSR A: the FP8 bytes come from the binned rows; S*A is formed only when
    # the solve escalates
    if kind == "csr":
        n, d = 20000, 32
        a = synth.csr_uniform(n, d, 0.2, seed=2)
        if cond > 1.0:
            a = (a @ sp.diags(np.logspace(0.0, -np.log10(cond), d))).tocsr()
        xt = np.random.default_rng(0).standard_normal(d)
        b = a @ xt + 1e-3 * np.random.default_rng(1).standard_normal(n)
    else:
        a, b, _ = synth.lsq_problem(20000, 32, cond, seed=2)
    x, info = api.lsq_solve(to_device(a), torch.from_numpy(b).cuda(), m=8 * 32, r=32 * 32,
                            seed=3, prec="fp8")
    _say(f"lsq fp8 {kind} cond={cond}: {info}")
    assert info["prec_used"] == want and info["status"] == "PSK_OK"
    rs, _ = olsq.lsq_quality(a, b, olsq.lstsq(a, b))
    rn, ne = olsq.lsq_quality(a, b, x.cpu().numpy())
    assert (rn - rs) / rs <= 1e-10 and ne <= 1e-10


def test_sketch_gcs_bf16_deterministic(api):
    a = to_device(synth.csr_uniform(50000, 200, 5e-3, seed=3))
    c1 = api.sketch_gcs(a, 150, 8000, seed=5, prec="bf16")
    c2 = api.sketch_gcs(a, 150, 8000, seed=5, prec="bf16")
    assert torch.equal(c1, c2)


@pytest.mark.parametrize("kind,cond,want", [("dense", 10.0, "bf16"), ("dense", 1e8, "f64"),
                                            ("csr", 1e2, "bf16"), ("csr", 1e8, "f64")])
def test_lsq_solve_bf16_sketch(api, kind, cond, want):
    # LSQR and the refinement run in FP64 whatever the sketch precision: the
    # solution meets the same tolerances as with the FP64 sketch.  An
    # ill-conditioned A makes the BF16 sketch escalate to FP64 (for CSR A the
    # BF16 limbs come from the binned rows, and S*A is formed only then).
    n, d = 20000, 32
    if kind == "csr":
        a = synth.csr_uniform(n, d, 0.2, seed=2)
        if cond > 1e2:
            # column scales spanning cond
            a = (a @ sp.diags(np.logspace(0.0, -np.log10(cond), d))).tocsr()
        xt = np.random.default_rng(0).standard_normal(d)
        b = a @ xt + 1e-3 * np.random.default_rng(1).standard_normal(n)
    else:
        a, b, _ = synth.lsq_problem(n, d, cond, seed=2)
    x, info = api.lsq_solve(to_device(a), torch.from_numpy(b).cuda(), m=4 * d, r=d * d,
                            seed=3, prec="bf16")
    _say(f"lsq bf16 {kind} cond={cond}: {info}")
    assert info["prec_used"] == want
    rs, _ = olsq.lsq_quality(a, b, olsq.lstsq(a, b))
    rn, ne = olsq.lsq_quality(a, b, x.cpu().numpy())
    assert (rn - rs) / rs <= 1e-10
    assert ne <= 1e-10
    assert info["status"] == "PSK_OK"


# ---------------------------------------------------------------------------
# Gram
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,n,d", [("dense", 20000, 50), ("dense", 3001, 130),
                                      ("csr", 100000, 500), ("csr", 20000, 70)])
def test_gram_f64(api, kind, n, d):
    _say(f"gram {kind} n={n} d={d}")
    a = synth.csr_uniform(n, d, 2e-3 if d > 100 else 0.05, seed=7) if kind == "csr" \
        else synth.dense_gaussian(n, d, seed=7)
    g = api.gram(to_device(a)).cpu().numpy()
    ref = og.gram(1.0, a)
    assert rel_fro(g, ref) <= 1e-13
    np.testing.assert_array_equal(g, g.T)


@pytest.mark.parametrize("n,d,dt,ld", [
    (7, 3, "f64", 3),           # fewer rows than one prefetch round
    (50000, 64, "f64", 64),     # one diagonal tile
    (10001, 65, "f64", 65),     # two tile rows, ragged column group (d % 4 = 1)
    (4001, 256, "f32", 256),    # the 4 x 4 tile triangle, FP32 vector loads
    (2000, 300, "f64", 301),    # odd row stride: scalar loads
    (3000, 130, "f32", 132),    # strided FP32 rows, ragged last tile
    (1, 1, "f64", 1)])
def test_gram_dense_shapes(api, n, d, dt, ld):
    """The slab SYRK: upper 64 x 64 tiles, diagonal tiles mirrored, rows and
    columns past the matrix read as zero, any row stride."""
    _say(f"gram dense n={n} d={d} {dt} ld={ld}")
    npdt = np.float64 if dt == "f64" else np.float32
    full = synth.dense_gaussian(n, ld, seed=8, dtype=npdt)
    a = full[:, :d]
    g = api.gram(to_device(full)[:, :d]).cpu().numpy().astype(np.float64)
    ref = og.gram(1.0, np.ascontiguousarray(a))
    assert rel_fro(g, ref) <= (1e-13 if dt == "f64" else 1e-6)
    np.testing.assert_array_equal(g, g.T)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_gram_integer_exact_and_alpha_beta(api, kind):
    a = synth.csr_integer(5000, 40, 0.1, seed=1) if kind == "csr" \
        else synth.dense_integer(5000, 40, seed=1)
    g = api.gram(to_device(a)).cpu().numpy()
    np.testing.assert_array_equal(g, og.gram(1.0, a))
    c0 = synth.dense_integer(40, 40, seed=2)
    c = to_device(c0)
    api.gram(to_device(a), alpha=2.0, beta=-3.0, C=c)
    np.testing.assert_array_equal(c.cpu().numpy(), og.gram(2.0, a, -3.0, c0))
    cn = torch.full((40, 40), float("nan"), dtype=torch.float64, device="cuda")
    api.gram(to_device(a), alpha=1.0, beta=0.0, C=cn)
    assert torch.isfinite(cn).all()


def test_gram_f32_input(api):
    a = synth.dense_gaussian(10000, 64, seed=3, dtype=np.float32)
    g = api.gram(to_device(a)).cpu().numpy().astype(np.float64)
    assert rel_fro(g, og.gram(1.0, a)) <= 1e-6


# ---------------------------------------------------------------------------
# squared row norms
# ---------------------------------------------------------------------------
def _rownorm_check(xh, a, b, alpha=1.0, beta=0.0, x0=None):
    ref = og.rownorms_sq(alpha, a, b, beta, x0)
    z = og.rownorm_bound_terms(a, b)
    nnz_row = a.getnnz(axis=1) if sp.issparse(a) else np.full(a.shape[0], a.shape[1])
    N = np.maximum(b.shape[1], nnz_row.max() ** 2) + a.shape[1] + 2
    bound = 3 * gamma(N, U64) * abs(alpha) * z + 1e-300
    if beta != 0.0:
        bound = bound + 2 * U64 * np.abs(beta * x0)
    assert np.all(np.abs(xh - ref) <= bound + 4 * U64 * np.abs(ref))


@pytest.mark.parametrize("kind,n,d,k", [("dense", 20000, 50, 50), ("dense", 5000, 130, 257),
                                        ("dense32", 7000, 256, 256), ("csr", 100000, 500, 500),
                                        ("csrzipf", 20000, 300, 64),
                                        # Zipf rows past max(32, k/8) entries as the
                                        # product a_i B, k above 1024 (8 columns a thread)
                                        ("csrzipf", 20000, 1200, 1500),
                                        ("csrzipf32", 20000, 900, 700),
                                        # ragged row tiles and k around the 64-column form
                                        ("dense", 9001, 70, 33), ("dense32", 3001, 256, 64),
                                        ("dense", 4097, 33, 65),
                                        # the LDS-resident column tile: 32-wide (k <= 32,
                                        # or d above 288), FP32 rows not in groups of 4;
                                        # and d beyond the LDS tile (the staged GEMM)
                                        ("dense", 5000, 40, 16), ("dense32", 3000, 400, 100),
                                        ("dense32", 2500, 254, 70), ("dense", 2000, 600, 70)])
def test_rownorms_sq(api, kind, n, d, k):
    _say(f"rownorms {kind} n={n} d={d} k={k}")
    if kind == "csr":
        a = synth.csr_uniform(n, d, 1e-3, seed=2)
    elif kind == "csrzipf":
        a = synth.csr_zipf(n, d, 1e-2, seed=2, dtype=np.float64)
    elif kind == "csrzipf32":
        a = synth.csr_zipf(n, d, 1e-2, seed=2, dtype=np.float32)
    elif kind == "dense32":
        a = synth.dense_gaussian(n, d, seed=2, dtype=np.float32)
    else:
        a = synth.dense_gaussian(n, d, seed=2)
    b = synth.dense_gaussian(d, k, seed=3)
    x = api.rownorms_sq(to_device(a), torch.from_numpy(b).cuda()).cpu().numpy()
    _rownorm_check(x, a, b)


@pytest.mark.parametrize("kind,n,d,k,shape", [
    ("dense32", 7000, 256, 256, "upper"),   # B = R^{-1}: paired tiles skip chunks
    ("dense", 5003, 200, 200, "upper"),     # ragged last tile, odd tile count
    ("dense", 4000, 96, 160, "band"),       # B zero below row 40: every tile short
    ("dense32", 3000, 128, 128, "lower"),   # full extent everywhere
    ("dense", 3000, 64, 64, "zerotile"),    # one 32-column tile of B all zero
    ("dense32", 3000, 400, 100, "upper"),   # single (unpaired) 32-column tiles
    ("dense", 2000, 70, 20, "upper"),       # k <= 32: one tile
    # zero lower-left quarters of the diagonal 32 x 32 blocks (16 x 16 block
    # upper triangular): the diagonal chunks skip them; one quarter holding
    # a nonzero (that tile takes its diagonal chunk whole)
    ("dense32", 7000, 256, 256, "upper16"), ("dense", 3000, 128, 128, "upper16"),
    ("dense", 5003, 200, 200, "quarterhit"), ("dense32", 3000, 400, 100, "upper16"),
    # FP32 rows read one element at a time (d % 4 != 0) with the diagonal
    # chunks, the last tile past d taken whole; B wider than d
    ("dense32", 2501, 254, 254, "upper"), ("dense32", 3000, 64, 160, "upper")])
def test_rownorms_sq_structured_b(api, kind, n, d, k, shape):
    """B with trailing zero rows per column (triangular, banded, zero tiles):
    the kernel skips the K chunks past each tile's extent, which must give
    the product's value (within the same bound as a full B)."""
    _say(f"rownorms structured {kind} n={n} d={d} k={k} {shape}")
    a = synth.dense_gaussian(n, d, seed=7, dtype=np.float32 if kind == "dense32"
                             else np.float64)
    b = synth.dense_gaussian(d, k, seed=8)
    if shape == "upper":
        b = np.triu(b)
    elif shape == "lower":
        b = np.tril(b)
    elif shape == "band":
        b[40:, :] = 0.0
    elif shape == "upper16":
        i, j = np.indices(b.shape)
        b[i // 16 > j // 16] = 0.0
    elif shape == "quarterhit":
        b = np.triu(b)
        b[32 * 2 + 20, 32 * 2 + 3] = 1.5
    else:
        b[:, 32:64] = 0.0
    x = api.rownorms_sq(to_device(a), torch.from_numpy(b).cuda()).cpu().numpy()
    _rownorm_check(x, a, b)


def test_rownorms_alpha_beta(api):
    a = synth.dense_gaussian(3000, 20, seed=4)
    b = synth.dense_gaussian(20, 20, seed=5)
    x0 = synth.dense_gaussian(3000, 1, seed=6)[:, 0]
    xd = torch.from_numpy(x0.copy()).cuda()
    api.rownorms_sq(to_device(a), torch.from_numpy(b).cuda(), alpha=0.5, beta=2.0, x=xd)
    _rownorm_check(xd.cpu().numpy(), a, b, 0.5, 2.0, x0)


def test_rownorms_alpha_beta_csr_long_rows(api):
    """alpha/beta on CSR rows of every form: one lane, one wavefront
    (quadratic form with B B^T) and the listed long rows (the product)."""
    a = synth.csr_zipf(6000, 300, 2e-2, seed=4, dtype=np.float64)
    assert a.getnnz(axis=1).max() > 300 // 8
    b = synth.dense_gaussian(300, 300, seed=5)
    x0 = synth.dense_gaussian(6000, 1, seed=6)[:, 0]
    xd = torch.from_numpy(x0.copy()).cuda()
    api.rownorms_sq(to_device(a), torch.from_numpy(b).cuda(), alpha=0.5, beta=2.0, x=xd)
    _rownorm_check(xd.cpu().numpy(), a, b, 0.5, 2.0, x0)


# ---------------------------------------------------------------------------
# QR of the sketch, leverage scores, least squares
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,d,cond", [(200, 50, 1e2), (1030, 257, 1e6), (96, 96, 1e3),
                                     (40, 1, 1.0), (64, 64, 10.0), (2000, 500, 1e8),
                                     (3000, 700, 1e4)])
def test_sketch_qr(api, m, d, cond):
    _say(f"sketch_qr m={m} d={d} cond={cond}")
    c, _, _ = synth.lsq_problem(m, d, cond, seed=1, noise=0.0)
    r, ri = api.sketch_qr(torch.from_numpy(c).cuda())
    r, ri = r.cpu().numpy(), ri.cpu().numpy()
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    # backward error of the factorization: R^T R = C^T C
    assert np.linalg.norm(r.T @ r - c.T @ c) / np.linalg.norm(c.T @ c) <= 1e-13
    ro = olev.qr_r(c)
    assert rel_fro(r, ro) <= 50 * cond * U64
    assert np.linalg.norm(ri @ r - np.eye(d)) <= 1e3 * cond * d * U64


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_leverage_pipeline(api, kind):
    n, d, m, r = (20000, 50, 200, 2500) if kind == "dense" else (100000, 64, 256, 8192)
    a = synth.dense_gaussian(n, d, seed=5) if kind == "dense" \
        else synth.csr_uniform(n, d, 0.05, seed=5)
    ad = to_device(a)
    c = api.sketch_gcs(ad, m, r, seed=9)
    _, ri = api.sketch_qr(c)
    th = api.rownorms_sq(ad, ri).cpu().numpy()
    tt, _ = olev.leverage_sketched(a, m, r, 9)
    # empty CSR rows have leverage exactly 0 on both sides
    assert np.all(np.abs(th - tt) <= 1e-9 * tt + 1e-300)
    # sketched leverage scores bracket the exact ones: with sigma the singular
    # values of G S Q (Q an orthonormal basis of range(A)),
    # theta_i / sigma_max^2 <= theta~_i <= theta_i / sigma_min^2
    ex = olev.leverage_exact(a)
    sv = olev.sketch_distortion(a, m, r, 9)
    tol = 1e-9 * ex + 1e-14
    assert np.all(th >= ex / sv.max() ** 2 - tol)
    assert np.all(th <= ex / sv.min() ** 2 + tol)


# Algorithm ls_approximate_drineas in one call, with and without the JL step.
# FP64 bar: R from the device's QR differs from LAPACK's by cond(C) u times a
# modest factor, so theta agrees to 1e-9 relative; FP32 A is exact in FP64
# and its S A is summed in FP64, so the same bar holds.
@pytest.mark.parametrize("kind,n,d,m,r,t", [
    ("dense", 20000, 50, 200, 2500, 0),
    ("dense", 20000, 50, 200, 2500, 16),
    ("dense", 20000, 50, 200, 2500, 100),    # t > 64 (wide row-norm tiles), t > d
    ("dense", 6000, 130, 0, 3001, 37),       # S A alone (m == 0), ragged t
    ("csr:0.02", 100000, 64, 256, 8192, 32),
    ("csr:0.02", 100000, 64, 0, 8192, 0),
    ("csr", 100000, 500, 640, 25000, 48),    # the sparse Gaussian product
    ("dense32", 8000, 96, 129, 1024, 24),
    ("dense32", 8000, 20, 0, 1024, 5),       # FP32 S A widened to FP64
    ("dense", 500, 1, 3, 7, 1)])             # d = 1, t = 1
def test_leverage_sketch_f64(api, kind, n, d, m, r, t):
    _say(f"leverage_sketch {kind} n={n} d={d} m={m} r={r} t={t}")
    a = _gcs_input(kind, n, d)
    th = api.leverage_sketch(to_device(a), m, r, seed=13, t=t).cpu().numpy()
    ref = olev.leverage_sketched_jl(a, m, r, t, 13)
    z = ref == 0
    assert np.array_equal(th[z], ref[z])  # empty rows: exactly 0
    err = np.abs(th[~z] / ref[~z] - 1).max()
    _say(f"  max rel err {err:.3e}, sum {th.sum():.6f}")
    assert err <= 1e-9


@pytest.mark.parametrize("dtype,t", [(np.float64, 0), (np.float64, 32), (np.float32, 0)])
def test_leverage_sketch_coherent(api, dtype, t):
    """The dense coherent structure (singular values geometric from 1 to 1e-6,
    5% of rows scaled by 100) at n = 100,000, d = 64.  The scores agree to
    ~cond(C) u for FP64 and for FP32 A alike (FP32 entries are exact in FP64
    and S A is summed in FP64)."""
    n, d, m, r = 100000, 64, 256, 4096
    a = synth.dense_coherent(n, d, seed=3, smin=1e-6, dtype=dtype)
    th = api.leverage_sketch(to_device(a), m, r, seed=1, t=t).cpu().numpy()
    ref = olev.leverage_sketched_jl(a, m, r, t, 1)
    err = np.abs(th / ref - 1)
    _say(f"leverage_sketch coherent {np.dtype(dtype).name} t={t}: max {err.max():.3e} "
         f"median {np.median(err):.3e}")
    assert err.max() <= 1e-7


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("kind,n,d,m,r,t", [
    ("dense", 20000, 50, 200, 2500, 16),
    ("csr:2e-3", 200000, 64, 256, 32768, 32)])
def test_leverage_sketch_reduced(api, prec, kind, n, d, m, r, t):
    """Against the oracle's scores from the quantised-operand sketch: the
    sketch's kernel arithmetic (normwise ~1e-6 BF16, <= 5e-4 FP8) times a
    small multiple of cond(C)."""
    _say(f"leverage_sketch {prec} {kind} n={n} d={d} m={m} r={r} t={t}")
    a = _gcs_input(kind, n, d)
    th = api.leverage_sketch(to_device(a), m, r, seed=13, t=t, prec=prec).cpu().numpy()
    q = osk.sketch_gcs_bf16_reference if prec == "bf16" else osk.sketch_gcs_fp8_reference
    ref = olev.leverage_from_sketch(a, q(a, m, r, 13), t, 13)
    z = ref == 0
    assert np.array_equal(th[z], ref[z])
    err = np.abs(th[~z] / ref[~z] - 1).max()
    _say(f"  max rel err vs quantised reference {err:.3e}")
    assert err <= (1e-3 if prec == "bf16" else 1e-2)


# ---------------------------------------------------------------------------
# the sketch perturbation delta = ||(C^ - C) R^{-1}||_2
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("kind,n,d,m,r", [
    ("dense", 20000, 50, 200, 2500),
    ("dense32", 8000, 96, 129, 1024),
    ("csr", 100000, 500, 640, 25000)])
def test_sketch_delta_vs_oracle(api, prec, kind, n, d, m, r):
    """The device delta of the device's reduced-precision sketch against the
    oracle's delta of the same two matrices (a lower estimate: never above,
    within 1e-6 relative here)."""
    a = _gcs_input(kind, n, d)
    ad = to_device(a)
    ch = api.sketch_gcs(ad, m, r, seed=5, prec=prec)
    c = api.sketch_gcs(ad, m, r, seed=5)
    dd = api.sketch_delta(ch, c).item()
    do = olev.sketch_perturbation(ch.cpu().numpy(), c.cpu().numpy())
    _say(f"sketch_delta {prec} {kind}: device {dd:.6e} oracle {do:.6e}")
    assert do * (1 - 1e-6) <= dd <= do * (1 + 1e-9)
    assert dd < 0.5


@pytest.mark.parametrize("m,d", [(5, 1), (7, 3), (2400, 1100)])
def test_sketch_delta_shapes(api, m, d):
    """delta at the size extremes (one column; a few; d above 1024 and not a
    multiple of 64, so several column blocks and several columns per
    thread in the choice of the dominant column) against the oracle's exact
    value, for C^ = C + E with a random E of relative size 1e-3."""
    rng = np.random.default_rng(m + d)
    c = rng.standard_normal((m, d))
    ch = c + 1e-3 * rng.standard_normal((m, d))
    dd = api.sketch_delta(torch.from_numpy(ch).cuda(), torch.from_numpy(c).cuda()).item()
    do = olev.sketch_perturbation(ch, c)
    _say(f"sketch_delta m={m} d={d}: device {dd:.9e} oracle {do:.9e}")
    assert do * (1 - 1e-6) <= dd <= do * (1 + 1e-9)


def test_sketch_delta_closed_forms(api):
    c = torch.from_numpy(osk.sketch_gcs(synth.dense_gaussian(4000, 30, seed=1), 90, 600, 2))
    c = c.cuda()
    assert api.sketch_delta(c, c).item() == 0.0
    assert api.sketch_delta(1.25 * c, c).item() == pytest.approx(0.25, rel=1e-12)


@pytest.mark.parametrize("prec,kind,n,d,m,r,smin", [
    ("bf16", "dense", 20000, 50, 200, 2500, None),
    ("fp8", "dense", 20000, 50, 200, 2500, None),
    ("bf16", "csr:2e-3", 200000, 64, 256, 32768, None),
    ("fp8", "csr:2e-3", 200000, 64, 256, 32768, None),
    ("bf16", "coherent", 100000, 64, 256, 4096, 1e-2),
    ("fp8", "coherent", 100000, 64, 256, 4096, 0.5)])
def test_leverage_reduced_within_delta_bracket(api, prec, kind, n, d, m, r, smin):
    """The validity bar for reduced-precision leverage scores: with delta of
    the device's sketch against the FP64 one, every score from the reduced
    sketch lies within |theta^ / theta~ - 1| <= (1 - delta)^-2 - 1 + 1e-10 of
    the oracle's FP64-sketch score (t = 0).  The cases keep delta < 1/2 (the
    FP8 sketch of the coherent matrix at cond 100 does not:
    test_fp8_delta_flags_ill_conditioned)."""
    a = (synth.dense_coherent(n, d, seed=3, smin=smin) if kind == "coherent"
         else _gcs_input(kind, n, d))
    ad = to_device(a)
    ch = api.sketch_gcs(ad, m, r, seed=13, prec=prec).cpu().numpy()
    c = osk.sketch_gcs(a, m, r, 13)
    delta = olev.sketch_perturbation(ch, c)
    th = api.leverage_sketch(ad, m, r, seed=13, t=0, prec=prec).cpu().numpy()
    ref = olev.leverage_sketched_jl(a, m, r, 0, 13)
    z = ref == 0
    assert np.array_equal(th[z], ref[z])
    err = np.abs(th[~z] / ref[~z] - 1).max()
    bound = olev.leverage_ratio_bound(delta) + 1e-10
    _say(f"leverage {prec} {kind}: delta {delta:.3e}, max |ratio - 1| {err:.3e}, "
         f"bound {bound:.3e}")
    assert delta < 0.5
    assert err <= bound


def test_fp8_delta_flags_ill_conditioned(api):
    """The FP8 sketch of the coherent matrix with singular values down to
    1e-2 (and 5% of rows scaled by 100) is no longer an embedding of A's
    column space: delta >= 1/2, where the scores of that sketch carry no
    guarantee; the FP64 and BF16 sketches stay far below."""
    n, d, m, r = 100000, 64, 256, 4096
    a = synth.dense_coherent(n, d, seed=3, smin=1e-2)
    ad = to_device(a)
    c = api.sketch_gcs(ad, m, r, seed=13)
    d8 = api.sketch_delta(api.sketch_gcs(ad, m, r, seed=13, prec="fp8"), c).item()
    d16 = api.sketch_delta(api.sketch_gcs(ad, m, r, seed=13, prec="bf16"), c).item()
    _say(f"coherent smin 1e-2: delta fp8 {d8:.3e}, bf16 {d16:.3e}")
    assert d8 >= 0.5 and d16 < 1e-2


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lsq_delta_est(api, prec):
    """lsq_solve with want_delta reports the delta of the sketch it
    preconditioned with; FP64 reports 0, no request NaN."""
    n, d, m, r = 20000, 32, 128, 1024
    a, b, _ = synth.lsq_problem(n, d, 10.0, seed=4)
    ad, bd = to_device(a), torch.from_numpy(b).cuda()
    x, info = api.lsq_solve(ad, bd, m=m, r=r, seed=3, prec=prec, want_delta=True)
    assert info["prec_used"] == prec
    ch = api.sketch_gcs(ad, m, r, seed=3, prec=prec).cpu().numpy()
    do = olev.sketch_perturbation(ch, osk.sketch_gcs(a, m, r, 3))
    _say(f"lsq {prec}: delta_est {info['delta_est']:.6e} oracle {do:.6e}")
    assert do * (1 - 1e-6) <= info["delta_est"] <= do * (1 + 1e-9)
    _, info64 = api.lsq_solve(ad, bd, m=m, r=r, seed=3, prec="f64", want_delta=True)
    assert info64["delta_est"] == 0.0
    _, info_n = api.lsq_solve(ad, bd, m=m, r=r, seed=3, prec=prec)
    assert np.isnan(info_n["delta_est"])
    rs, _ = olsq.lsq_quality(a, b, olsq.lstsq(a, b))
    rn, ne = olsq.lsq_quality(a, b, x.cpu().numpy())
    assert (rn - rs) / rs <= 1e-10 and ne <= 1e-10


def test_leverage_sketch_matches_composed_calls(api):
    """t = 0 is sketch_gcs, sketch_qr and rownorms_sq in sequence, bit for bit."""
    a = to_device(synth.csr_uniform(100000, 64, 0.05, seed=5))
    th = api.leverage_sketch(a, 256, 8192, seed=9, t=0, prec="bf16")
    _, ri = api.sketch_qr(api.sketch_gcs(a, 256, 8192, seed=9, prec="bf16"))
    assert torch.equal(th, api.rownorms_sq(a, ri))


def test_leverage_sketch_reports_rank_deficiency(api):
    a = synth.dense_gaussian(3000, 12, seed=1)
    a[:, 7] = 0.0
    with pytest.raises(RuntimeError, match="rank|ERANK"):
        api.leverage_sketch(to_device(a), 0, 400, seed=2, t=4)
        torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Column subset selection (Algorithm cgrrqr) and Algorithm ls_hrn_exact
# ---------------------------------------------------------------------------
def _css_input(kind, n, d, spread):
    """_gcs_input with its columns scaled by a permuted geometric sequence
    from 1 to 1/spread (spread 1: unscaled), so that the pivots have margins."""
    a = _gcs_input(kind, n, d)
    if spread == 1:
        return a
    sc = np.logspace(0, -np.log10(spread), d)[np.random.default_rng(3).permutation(d)]
    if sp.issparse(a):
        return (a @ sp.diags(sc)).tocsr().astype(a.dtype)
    return (a * sc).astype(a.dtype)


def _check_pivots(dev, b, k, tol):
    """dev equals the oracle's pivots, or (near ties) is a valid outcome: at
    every step the column taken has the largest residual norm up to tol."""
    ref, _ = ocss.qrcp_pivots(b, k)
    assert len(set(dev.tolist())) == k and dev.min() >= 0 and dev.max() < b.shape[1]
    if np.array_equal(dev, ref):
        return 0
    took, best = ocss.qrcp_replay(b, dev)
    assert np.all(took >= best * (1 - tol)), (dev, ref)
    return int(np.argmax(dev != ref))


@pytest.mark.parametrize("kind,n,d,m,r,k,spread", [
    ("dense", 20000, 50, 200, 2500, 50, 100.0),    # all d pivots
    ("dense", 20000, 50, 100, 2500, 20, 1.0),      # unscaled: near ties allowed
    ("dense", 6000, 130, 0, 3001, 40, 1e3),        # S A alone (m == 0)
    ("csr:0.02", 100000, 64, 256, 8192, 20, 10.0),
    ("csr", 100000, 500, 1000, 25000, 100, 1e3),   # m = 2d (the algorithm's choice)
    ("dense32", 8000, 96, 200, 1024, 96, 1e2),
    ("dense", 500, 1, 3, 7, 1, 1.0)])              # d = 1
def test_css_select(api, kind, n, d, m, r, k, spread):
    _say(f"css_select {kind} n={n} d={d} m={m} r={r} k={k} spread={spread}")
    a = _css_input(kind, n, d, spread)
    dev = api.css_select(to_device(a), m, r, k, seed=17).cpu().numpy().astype(np.int64)
    b = osk.sketch_gcs(a, m, r, 17)
    first = _check_pivots(dev, b, k, 1e-10)
    _say(f"  pivots equal to the oracle's up to step {first or k}")
    if spread > 1:
        assert first == 0


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_css_select_reduced(api, prec):
    a = _css_input("dense", 20000, 50, 1e2)
    dev = api.css_select(to_device(a), 200, 2500, 30, seed=17, prec=prec).cpu().numpy()
    q = osk.sketch_gcs_bf16_reference if prec == "bf16" else osk.sketch_gcs_fp8_reference
    _check_pivots(dev.astype(np.int64), q(a, 200, 2500, 17), 30, 1e-3)


def test_css_select_zero_columns_last(api):
    a = synth.dense_gaussian(5000, 12, seed=3)
    a[:, [2, 9]] = 0.0
    dev = api.css_select(to_device(a), 48, 600, 12, seed=1).cpu().numpy()
    np.testing.assert_array_equal(dev[10:], [2, 9])


@pytest.mark.parametrize("kind,n,d,m,r,k", [
    ("dense", 20000, 50, 100, 2500, 50),     # k = d: the exact scores of A
    ("dense", 20000, 50, 100, 2500, 12),
    ("csr:0.02", 100000, 64, 128, 8192, 30),
    ("csr", 100000, 500, 1000, 25000, 100),
    ("dense32", 8000, 96, 200, 1024, 40)])
def test_leverage_css(api, kind, n, d, m, r, k):
    _say(f"leverage_css {kind} n={n} d={d} m={m} r={r} k={k}")
    a = _css_input(kind, n, d, 100.0)
    th, cols = api.leverage_css(to_device(a), m, r, k, seed=5)
    ref, rcols = ocss.leverage_css(a, m, r, k, 5)
    np.testing.assert_array_equal(cols.cpu().numpy(), rcols)
    th = th.cpu().numpy()
    # the Gram route: cond(A[:, K])^2 u, cond <= ~1e2 here (column spread)
    err = np.abs(th - ref).max()
    _say(f"  max |dtheta| {err:.3e}, sum {th.sum():.10f}")
    assert err <= 1e-8
    assert abs(th.sum() - k) <= 1e-8 * k
    if k == d:
        assert np.abs(th - olev.leverage_exact(a)).max() <= 1e-8


def test_leverage_css_reports_rank_deficiency(api):
    a = synth.dense_gaussian(3000, 10, seed=2)
    a[:, 4] = 0.0
    with pytest.raises(RuntimeError, match="rank|ERANK"):
        api.leverage_css(to_device(a), 40, 500, 10, seed=1)
        torch.cuda.synchronize()


def test_lsq_solve_with_precomputed_preconditioner(api):
    a, b, _ = synth.lsq_problem(20000, 40, 1e5, seed=4)
    ad = to_device(a)
    _, ri = api.sketch_qr(api.sketch_gcs(ad, 160, 1600, seed=1))
    x, info = api.lsq_solve(ad, torch.from_numpy(b).cuda(), Rinv=ri)
    rs, _ = olsq.lsq_quality(a, b, olsq.lstsq(a, b))
    rn, ne = olsq.lsq_quality(a, b, x.cpu().numpy())
    assert (rn - rs) / rs <= 1e-10 and ne <= 1e-10 and info["status"] == "PSK_OK"


def test_kernel_timing_records_launches(api):
    a = to_device(synth.dense_gaussian(5000, 64, seed=1))
    with api.kernel_timing() as kt:
        api.sketch_gcs(a, 64, 512, seed=2)
        torch.cuda.synchronize()
        st = kt.stats()
    assert st["gauss_gemm"][1] == 1 and st["gauss_gemm"][0] > 0
    assert st["cs_scatter"][1] == 1 and st["cs_bin"][1] == 1


@pytest.mark.parametrize("kind,n,d,cond,r", [
    ("dense", 20000, 32, 1e3, None), ("dense", 20000, 32, 1e8, None),
    ("csr", 20000, 32, 1e2, None),
    # the dense pass's row batches: eight rows a wavefront (d <= 64, n >=
    # 65,536; ragged n), and the widths past 256 columns (two rows)
    ("dense", 100003, 48, 1e6, None), ("dense", 30001, 300, 1e3, 2400),
    ("dense", 20000, 600, 1e2, 4800)])
def test_lsq_solve_matches_lapack(api, kind, n, d, cond, r):
    _say(f"lsq {kind} n={n} d={d} cond={cond:g}")
    if kind == "csr":
        a = synth.csr_uniform(n, d, 0.2, seed=2)
        xt = np.random.default_rng(0).standard_normal(d)
        b = a @ xt + 1e-3 * np.random.default_rng(1).standard_normal(n)
    else:
        a, b, _ = synth.lsq_problem(n, d, cond, seed=2)
    x, info = api.lsq_solve(to_device(a), torch.from_numpy(b).cuda(), m=4 * d,
                            r=d * d if r is None else r, seed=3)
    _say(f"lsq {kind} cond={cond}: {info}")
    x = x.cpu().numpy()
    xs = olsq.lstsq(a, b)
    rs, _ = olsq.lsq_quality(a, b, xs)
    rn, ne = olsq.lsq_quality(a, b, x)
    assert (rn - rs) / rs <= 1e-10
    assert ne <= 1e-10
    assert info["status"] == "PSK_OK"


# ---------------------------------------------------------------------------
# Direct solvers and exact leverage scores (Gram route; sketch-and-solve)
# ---------------------------------------------------------------------------
def _direct_input(kind, cond):
    if kind == "csr":
        return synth.csr_uniform(100000, 64, 0.02, seed=4)
    if kind == "csr32":
        return synth.csr_uniform(50000, 48, 0.05, seed=4, dtype=np.float32)
    if kind == "dense32":
        return synth.dense_gaussian(20000, 40, seed=4, dtype=np.float32)
    a, _, _ = synth.lsq_problem(20000, 40, cond, seed=4)
    return a


@pytest.mark.parametrize("kind,cond", [("dense", 1.0), ("dense", 1e3), ("csr", 1.0),
                                       ("csr32", 1.0), ("dense32", 1.0)])
def test_leverage_gram_exact(api, kind, cond):
    a = _direct_input(kind, cond)
    d = a.shape[1]
    th = api.leverage_gram(to_device(a)).cpu().numpy()
    ex = olev.leverage_exact(a)
    err = np.abs(th - ex).max()
    _say(f"leverage_gram {kind} cond={cond}: max |dtheta| {err:.3e}, sum {th.sum():.12f}")
    # B = A^T A carries cond^2: the scores are exact to about cond^2 u
    tol = 1e-12 * max(cond, 1.0) ** 2
    assert err <= tol
    assert abs(th.sum() - d) <= d * tol


def test_leverage_gram_reports_rank_deficiency(api):
    a = synth.dense_gaussian(3000, 12, seed=1)
    a[:, 5] = 0.0  # a zero column: a zero pivot
    with pytest.raises(RuntimeError, match="rank|ERANK"):
        api.leverage_gram(to_device(a))
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind,cond", [("dense", 1.0), ("dense", 1e3), ("csr", 1.0),
                                       ("dense32", 1.0)])
def test_lsq_gram_matches_lapack(api, kind, cond):
    a = _direct_input(kind, cond)
    n = a.shape[0]
    rng = np.random.default_rng(7)
    b = a @ rng.standard_normal(a.shape[1]) + 1e-3 * rng.standard_normal(n)
    b = np.asarray(b, dtype=np.float64)
    x = api.lsq_gram(to_device(a), torch.from_numpy(b).cuda()).cpu().numpy()
    xs = olsq.lstsq(a, b)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    _say(f"lsq_gram {kind} cond={cond}: rel err {err:.3e}")
    assert err <= 1e-12 * max(cond, 1.0) ** 2


@pytest.mark.parametrize("kind,n,d,m,r", [
    ("dense", 20000, 32, 128, 1024),
    ("csr", 100000, 64, 256, 8192),           # S*A dense enough for the GEMM
    ("csr:2e-3", 200000, 64, 256, 32768)])    # the product over S*A's nonzeros
@pytest.mark.parametrize("prec", ["f64", "bf16", "fp8"])
def test_lsq_sketch_solve(api, kind, n, d, m, r, prec):
    if kind == "dense":
        a, b, _ = synth.lsq_problem(n, d, 10.0, seed=8)
    else:
        dens = float(kind.split(":")[1]) if ":" in kind else 0.02
        a = synth.csr_uniform(n, d, dens, seed=8)
        rng = np.random.default_rng(2)
        b = a @ rng.standard_normal(d) + 1e-2 * rng.standard_normal(n)
    b = np.asarray(b, dtype=np.float64)
    x = api.lsq_sketch_solve(to_device(a), torch.from_numpy(b).cuda(), m, r, seed=11,
                             prec=prec).cpu().numpy()
    if prec == "f64":
        ref = olsq.lsq_sketch_solve(a, b, m, r, 11)
        tol = 1e-10
    else:
        q = (osk.sketch_gcs_bf16_reference if prec == "bf16" else osk.sketch_gcs_fp8_reference)
        c = q(a, m, r, 11)
        cb = q(b[:, None], m, r, 11)[:, 0]
        ref = olsq.lstsq(c, cb)
        # the sketch's kernel arithmetic (~2e-5 BF16, ~5e-4 FP8 normwise)
        # times cond(A~) ~ 10
        tol = 5e-4 if prec == "bf16" else 5e-3
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    # the residual of the sketched solution against the optimum (1 + d/m-ish)
    xs = olsq.lstsq(a, b)
    ratio = np.linalg.norm(a @ x - b) / np.linalg.norm(a @ xs - b)
    _say(f"lsq_sketch_solve {prec} {kind}: vs reference {err:.3e}, residual ratio {ratio:.4f}")
    assert err <= tol
    assert ratio >= 1.0 - 1e-12
    if prec != "fp8":
        # FP8's ~5% operand rounding moves the sketched solution by more than
        # the optimal residual of these near-consistent problems; its bar is
        # the quantised reference above
        assert ratio <= 1.0 + 4.0 * d / m
