"""OSNAP with s > 1 non-zeros per column on the device against the oracle
(oracle/osnap.py): the hash bit for bit, S*A and G*S*A in every precision on
dense and CSR input across tiles, ragged tails and the split-bucket path,
s = 1 identical to the CountSketch calls, and leverage scores from an OSNAP
sketch on a coherent matrix that CountSketch of the same size cannot embed."""
import numpy as np
import pytest

import synth
from helpers import gamma, rel_fro, to_device
from oracle import leverage as olev
from oracle import osnap as oo
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


@pytest.mark.parametrize("n,r,s,row0", [(100_000, 65536, 4, 0), (5000, 105, 7, 2 ** 33 + 5),
                                        (20000, 512, 512, 0), (3, 8, 2, 0)])
def test_osnap_hash_bit_exact(api, n, r, s, row0):
    _say(f"osnap_hash n={n} r={r} s={s} row0={row0}")
    h, sg = api.osnap_hash(n, s, r, seed=12345, row0=row0)
    ho, so = oo.osnap_hash(n, r, s, seed=12345, row0=row0)
    np.testing.assert_array_equal(h.cpu().numpy().astype(np.int64), ho)
    np.testing.assert_array_equal(sg.cpu().numpy(), so)


def test_osnap_s1_is_countsketch(api):
    h, sg = api.osnap_hash(50000, 1, 777, seed=3)
    h1, s1 = api.cs_hash(50000, 777, seed=3)
    assert torch.equal(h[:, 0], h1) and torch.equal(sg[:, 0], s1)
    a = to_device(synth.dense_gaussian(30001, 37, seed=1))
    assert torch.equal(api.sketch_osnap(a, 1, 0, 1024, 5), api.sketch_cs(a, 1024, 5))
    for prec in ("f64", "bf16", "fp8"):
        assert torch.equal(api.sketch_osnap(a, 1, 96, 1024, 5, prec=prec),
                           api.sketch_gcs(a, 96, 1024, 5, prec=prec))


def _bound_ok(got, ref, mag, k, out_u):
    """|got - ref| <= out_u |ref| + 2 gamma_k mag (the FP64 sum of at most k
    signed terms, one product by 1/sqrt(s), one rounding to the output)."""
    u = 2.0 ** -53
    return np.all(np.abs(got - ref) <= out_u * np.abs(ref) + 2 * gamma(k + 2, u) * mag)


@pytest.mark.parametrize("kind,dtype,n,d,r,s", [
    ("dense", np.float64, 30001, 37, 1024, 2),
    ("dense", np.float32, 30001, 37, 1536, 3),
    ("dense", np.float64, 20000, 300, 4096, 8),      # several column groups per lane
    ("dense", np.float64, 200_000, 9, 64, 4),        # long buckets: split + combine
    ("dense", np.float32, 200_000, 9, 64, 4),
    ("csr", np.float64, 50000, 70, 2048, 4),
    ("csr", np.float32, 50000, 70, 2048, 8),
    ("csr", np.float64, 300_000, 20, 32, 2),         # CSR split + combine
])
def test_sketch_osnap_sa(api, kind, dtype, n, d, r, s):
    _say(f"S*A osnap {kind} {np.dtype(dtype).name} n={n} d={d} r={r} s={s}")
    a = (synth.csr_uniform(n, d, 0.05, seed=2, dtype=dtype) if kind == "csr"
         else synth.dense_gaussian(n, d, seed=2).astype(dtype))
    got = api.sketch_osnap(to_device(a), s, 0, r, seed=7)
    assert got.dtype == (torch.float64 if dtype == np.float64 else torch.float32)
    got = got.double().cpu().numpy()
    ref = oo.sketch_osnap(a, r, s, 7)
    S = oo.osnap_sparse(n, r, s, 7)
    mag = abs(S) @ abs(a.astype(np.float64))
    mag = mag.toarray() if hasattr(mag, "toarray") else np.asarray(mag)
    longest = int(np.bincount(oo.osnap_hash(n, r, s, 7)[0].ravel(), minlength=r).max())
    out_u = 0.0 if dtype == np.float64 else 2.0 ** -24
    assert _bound_ok(got, ref, mag, longest, out_u)


@pytest.mark.parametrize("kind,s", [("dense", 4), ("csr", 8)])
def test_sketch_osnap_gaussian(api, kind, s):
    n, d, r, m = 40000, 48, 4096, 160
    a = (synth.csr_uniform(n, d, 0.03, seed=4) if kind == "csr"
         else synth.dense_gaussian(n, d, seed=4))
    A = to_device(a)
    sa = oo.sketch_osnap(a, r, s, 9)
    ref64 = oo.sketch_gosnap(a, m, r, s, 9)
    for prec, tol in (("f64", 1e-13), ("bf16", 1e-4), ("fp8", 1e-4)):
        _say(f"G S A osnap {kind} s={s} {prec}")
        c = api.sketch_osnap(A, s, m, r, seed=9, prec=prec).cpu().numpy()
        if prec == "f64":
            ref = ref64
        elif prec == "bf16":
            ref = osk.gauss_product_bf16_reference(sa, m, 9)
        else:
            ref = osk.gauss_product_fp8_reference(sa, m, 9)
        e = rel_fro(c, ref)
        _say(f"  vs its definition {e:.3e}")
        assert e <= tol
        if prec != "f64":
            assert rel_fro(c, ref64) <= (1e-2 if prec == "bf16" else 1e-1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sketch_osnap_gaussian_over_nonzeros(api, dtype):
    """CSR A whose OSNAP S*A is sparse (s nnz(A) at most r d / 32): the FP64
    and BF16 Gaussian products run over the nonzeros of S*A, formed from the
    OSNAP's bins with 1/sqrt(s) applied to each bucket sum (FP8 keeps its
    dense form above r d / 512); every precision against its definition
    (FP64 to 1e-13, BF16 and FP8 against the quantised references at
    1e-4)."""
    n, d, r, m, s = 200_000, 64, 65536, 96, 4
    a = synth.csr_uniform(n, d, 1e-3, seed=12, dtype=dtype)
    assert a.nnz * s * 32 <= r * d
    A = to_device(a)
    sa = oo.sketch_osnap(a, r, s, 3)
    ref64 = oo.sketch_gosnap(a, m, r, s, 3)
    for prec, tol in (("f64", 1e-13), ("bf16", 1e-4), ("fp8", 1e-4)):
        c = api.sketch_osnap(A, s, m, r, seed=3, prec=prec).cpu().numpy()
        ref = {"f64": ref64, "bf16": osk.gauss_product_bf16_reference(sa, m, 3),
               "fp8": osk.gauss_product_fp8_reference(sa, m, 3)}[prec]
        e = rel_fro(c, ref)
        _say(f"G S A osnap over nonzeros {np.dtype(dtype).name} {prec}: {e:.3e}")
        assert e <= tol


def test_osnap_leverage_on_coherent_rows(api):
    """d rows of leverage 1 (scaled identity rows) inside a Gaussian block,
    r = 8 d: the scores from S*A with OSNAP s = 8 match the oracle's scores
    from the same sketch, and stay within the embedding bracket of the exact
    ones, where the CountSketch of the same size collapses."""
    rng = np.random.default_rng(6)
    n, d = 20000, 32
    r = 8 * d
    a = rng.standard_normal((n, d)) * 1e-3
    a[:d] += 10.0 * np.eye(d)
    A = to_device(a)
    exact = olev.leverage_exact(a)
    ok_runs = 0
    for seed in range(4):
        c = api.sketch_osnap(A, 8, 0, r, seed=seed)
        _, ri = api.sketch_qr(c)
        th = api.rownorms_sq(A, ri).cpu().numpy()
        want = olev.leverage_from_sketch(a, oo.sketch_osnap(a, r, 8, seed), 0, seed)
        assert rel_fro(th, want) <= 1e-9
        sv = np.linalg.svd(oo.sketch_osnap(np.linalg.qr(a)[0], r, 8, seed), compute_uv=False)
        eps = max(sv.max() - 1, 1 - sv.min())
        assert eps < 0.8
        ratio = th[:d] / exact[:d]
        assert ratio.min() >= (1 + eps) ** -2 * (1 - 1e-9)
        assert ratio.max() <= (1 - eps) ** -2 * (1 + 1e-9)
        ok_runs += 1
    assert ok_runs == 4


def test_osnap_argument_checks(api):
    from paper_2203_02798_amd import _lib as L
    a = to_device(synth.dense_gaussian(1000, 8, seed=0))
    for s, r in ((0, 64), (3, 64), (65, 64)):
        with pytest.raises(L.PskError) as e:
            api.sketch_osnap(a, s, 0, r, seed=1)
        assert e.value.status == L.PSK_EINVAL
    with pytest.raises(L.PskError):
        api.osnap_hash(10, 3, 64, seed=1)
