"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/psk.h declares, plans workspaces, and rejects bad
arguments with the documented status codes before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2203_02798_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "psk.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libpsk.so is not built; run `python -m paper_2203_02798_amd.build`")
    return L.lib()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert set(declared) == set(L.EXPORTED), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version(lib):
    assert b"gfx950" in lib.psk_version()


def _dense(n, d, dtype=L.PSK_F64, ld=None):
    m = L.PskMat()
    m.format, m.dtype, m.n, m.d = L.PSK_DENSE, dtype, n, d
    m.ld = ld if ld is not None else d
    m.values = 0x1000  # never dereferenced by planning/validation
    return m


def _csr(n, d, nnz):
    m = L.PskMat()
    m.format, m.dtype, m.n, m.d, m.ld, m.nnz = L.PSK_CSR, L.PSK_F64, n, d, d, nnz
    m.values, m.indptr, m.indices = 0x1000, 0x2000, 0x3000
    return m


def _ws(op, mat, m=0, r=1, k=1, prec=0):
    out = ctypes.c_size_t(0)
    st = L.lib().psk_workspace_size(op, ctypes.byref(mat), m, r, k, prec, ctypes.byref(out))
    return st, out.value


def test_workspace_planning(lib):
    st, b1 = _ws(L.PSK_OP_SKETCH_CS, _dense(20000, 50), r=2500)
    assert st == 0 and b1 >= 20000 * 4 * 2
    st, b2 = _ws(L.PSK_OP_SKETCH_GCS, _dense(20000, 50), m=200, r=2500)
    assert st == 0 and b2 > b1 + 2500 * 50 * 8
    # sparse S*A (500,000 nonzeros in 250,000 x 500): the product runs over its
    # nonzeros, which are staged (slot, column, value) instead of the r x d array
    st, b3 = _ws(L.PSK_OP_SKETCH_GCS, _csr(1_000_000, 500, 500_000), m=2000, r=250_000)
    assert st == 0 and 500_000 * 16 <= b3 < 250_000 * 500 * 8
    # a denser CSR matrix takes the GEMM, with S*A staged in the workspace
    st, b3d = _ws(L.PSK_OP_SKETCH_GCS, _csr(100_000, 64, 3_000_000), m=256, r=8192)
    assert st == 0 and b3d > 8192 * 64 * 8
    st, b4 = _ws(L.PSK_OP_GRAM, _dense(1000, 64))
    assert st == 0 and b4 > 0
    st, b5 = _ws(L.PSK_OP_ROWNORMS, _csr(1000, 64, 100), k=64)
    assert st == 0 and b5 >= 64 * 64 * 8
    q = L.PskMat(); q.n, q.d = 400, 100
    st, b6 = _ws(L.PSK_OP_QR, q)
    assert st == 0 and b6 >= 2 * 400 * 100 * 8
    st, b7 = _ws(L.PSK_OP_LSQ, _dense(5000, 32), m=128, r=1024)
    assert st == 0 and b7 > 5000 * 8
    # with want_delta (k != 0) a BF16 solve also holds the FP64 sketch and its
    # factor; an FP64 solve has nothing to compare
    st, b7d = _ws(L.PSK_OP_LSQ, _dense(5000, 32), m=128, r=1024, k=1, prec=L.PSK_PREC_BF16)
    st2, b7b = _ws(L.PSK_OP_LSQ, _dense(5000, 32), m=128, r=1024, k=0, prec=L.PSK_PREC_BF16)
    assert st == 0 and st2 == 0 and b7d >= b7b + 2 * 128 * 32 * 8
    q2 = L.PskMat(); q2.n, q2.d = 128, 32
    st, bd = _ws(L.PSK_OP_DELTA, q2)
    assert st == 0 and bd >= 2 * 128 * 32 * 8
    q2.n = 16
    st, _ = _ws(L.PSK_OP_DELTA, q2)
    assert st == -1  # m < d
    st, b8 = _ws(L.PSK_OP_LSQ, _dense(5000, 32), m=0, r=0)  # caller's own R^{-1}
    assert st == 0 and 5000 * 8 < b8 < b7
    st, _ = _ws(L.PSK_OP_LSQ, _dense(5000, 32), m=16, r=1024)  # m < d
    assert st == -1
    st, _ = _ws(L.PSK_OP_SKETCH_CS, _dense(5000, 32), r=0)
    assert st == -1
    # G*A: dense A is the GEMM operand in place (a contiguous copy when
    # ld > d); CSR A stages its entries and one bin per row
    st, g1 = _ws(L.PSK_OP_SKETCH_G, _dense(20000, 50), m=200)
    assert st == 0 and g1 < 20000 * 50 * 8
    st, g2 = _ws(L.PSK_OP_SKETCH_G, _dense(20000, 50, ld=64), m=200)
    assert st == 0 and g2 >= g1 + 20000 * 50 * 8
    st, g3 = _ws(L.PSK_OP_SKETCH_G, _csr(1_000_000, 500, 500_000), m=1000)
    assert st == 0 and g3 >= 500_000 * 28 + 2 * 1_000_000 * 4
    st, _ = _ws(L.PSK_OP_SKETCH_G, _csr(1000, 2000, 100), m=10)
    assert st == -7  # CSR with d > 1023
    st, _ = _ws(L.PSK_OP_SKETCH_G, _dense(100, 5), m=0)
    assert st == -1
    # direct solvers: the FP64 Gram matrix, its factor and inverse (d x d each)
    st, l1 = _ws(L.PSK_OP_LEVERAGE_GRAM, _csr(100_000, 200, 10_000))
    assert st == 0 and l1 >= 3 * 200 * 200 * 8
    st, l2 = _ws(L.PSK_OP_LSQ_GRAM, _dense(5000, 64))
    assert st == 0 and l2 >= 3 * 64 * 64 * 8
    st, l3 = _ws(L.PSK_OP_LSQ_SKETCH, _dense(5000, 64), m=256, r=1024)
    assert st == 0 and l3 >= 256 * 64 * 8
    st, _ = _ws(L.PSK_OP_LSQ_SKETCH, _dense(5000, 64), m=32, r=1024)  # m < d
    assert st == -1
    st, _ = _ws(L.PSK_OP_LEVERAGE_GRAM, _dense(50000, 5000))
    assert st == -7  # d > 4096
    # sketched leverage: the sketch (m x d, or r x d for S A alone), two
    # copies for the QR passes; the JL step adds Pi and R^{-1} Pi (d x t each)
    st, s1 = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=200, r=2500, k=0)
    assert st == 0 and s1 >= 3 * 200 * 50 * 8
    st, s2 = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=200, r=2500, k=16)
    assert st == 0 and s2 >= s1
    st, s3 = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=0, r=2500, k=0)
    assert st == 0 and s3 >= 3 * 2500 * 50 * 8
    st, _ = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=0, r=40)  # r < d
    assert st == -1
    st, _ = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=30, r=2500)  # m < d
    assert st == -1
    st, _ = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=64, r=2500, k=-1)
    assert st == -1
    st, _ = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=64, r=2500, prec=4)
    assert st == -2
    st, _ = _ws(L.PSK_OP_LEVERAGE_SKETCH, _dense(20000, 50), m=0, r=2500, prec=4)
    assert st == 0  # prec is not read without the Gaussian stage
    # column subset selection: the sketch and its column-major copy; the
    # leverage scores add the d x d Gram matrix
    st, c1 = _ws(L.PSK_OP_CSS, _dense(20000, 50), m=100, r=2500, k=10)
    assert st == 0 and c1 >= 2 * 100 * 50 * 8
    st, c2 = _ws(L.PSK_OP_LEVERAGE_CSS, _dense(20000, 50), m=100, r=2500, k=10)
    assert st == 0 and c2 >= c1 + 50 * 50 * 8
    for k in (0, 51):
        st, _ = _ws(L.PSK_OP_CSS, _dense(20000, 50), m=100, r=2500, k=k)
        assert st == -1
    st, _ = _ws(L.PSK_OP_CSS, _csr(1000, 5000, 100), m=6000, r=8000, k=3)
    assert st == -7  # d > 4096


def test_rejects_bad_arguments_without_device_work(lib):
    stream = None
    sa = ctypes.c_void_p(0x4000)
    ws = ctypes.c_void_p(0x5000)
    assert lib.sketch_cs(None, 10, 0, sa, ws, 1 << 20, stream) == -1
    bad = _dense(10, 5)
    assert lib.sketch_cs(ctypes.byref(bad), 0, 0, sa, ws, 1 << 20, stream) == -1
    assert b"r must be" in lib.psk_last_error()
    bad.ld = 3
    assert lib.sketch_cs(ctypes.byref(bad), 4, 0, sa, ws, 1 << 20, stream) == -1
    bad = _dense(10, 5, dtype=7)
    assert lib.sketch_cs(ctypes.byref(bad), 4, 0, sa, ws, 1 << 20, stream) == -2
    good = _dense(10, 5)
    assert lib.sketch_cs(ctypes.byref(good), 4, 0, sa, ws, 16, stream) == -3
    assert lib.sketch_gcs(ctypes.byref(good), -1, 4, 0, 0, sa, ws, 1 << 20, stream) == -1
    assert lib.sketch_gcs(ctypes.byref(good), 3, 4, 0, 9, sa, ws, 1 << 20, stream) == -2
    assert lib.sketch_g(ctypes.byref(good), 0, 0, 0, sa, ws, 1 << 20, stream) == -1
    assert lib.sketch_g(ctypes.byref(good), 3, 0, 5, sa, ws, 1 << 20, stream) == -2
    assert lib.sketch_g(ctypes.byref(good), 3, 0, 0, None, ws, 1 << 20, stream) == -1
    assert lib.sketch_g(ctypes.byref(good), 3, 0, 0, sa, ws, 16, stream) == -3
    assert lib.leverage_gram(ctypes.byref(good), None, ws, 1 << 20, stream) == -1
    assert lib.leverage_gram(ctypes.byref(good), sa, ws, 16, stream) == -3
    assert lib.lsq_gram(ctypes.byref(good), None, sa, ws, 1 << 20, stream) == -1
    assert lib.lsq_sketch_solve(ctypes.byref(good), sa, sa, 4, 8, 0, 0, ws, 1 << 20,
                                stream) == -1  # m < d
    assert lib.lsq_sketch_solve(ctypes.byref(good), sa, sa, 8, 16, 0, 3, ws, 1 << 20,
                                stream) == -2  # prec
    assert lib.leverage_sketch(ctypes.byref(good), 8, 16, 0, 0, 0, None, ws, 1 << 20,
                               stream) == -1  # theta
    assert lib.leverage_sketch(ctypes.byref(good), 4, 16, 0, 0, 0, sa, ws, 1 << 20,
                               stream) == -1  # m < d
    assert lib.leverage_sketch(ctypes.byref(good), 0, 4, 0, 0, 0, sa, ws, 1 << 20,
                               stream) == -1  # m == 0 and r < d
    assert lib.leverage_sketch(ctypes.byref(good), 8, 16, 0, 0, 7, sa, ws, 1 << 20,
                               stream) == -2  # prec
    assert lib.leverage_sketch(ctypes.byref(good), 8, 16, 4, 0, 0, sa, ws, 16,
                               stream) == -3  # workspace
    assert lib.css_select(ctypes.byref(good), 8, 16, 3, 0, 0, None, ws, 1 << 20,
                          stream) == -1  # cols
    assert lib.css_select(ctypes.byref(good), 8, 16, 6, 0, 0, sa, ws, 1 << 20,
                          stream) == -1  # k > d
    assert lib.css_select(ctypes.byref(good), 8, 16, 3, 0, 0, sa, ws, 16, stream) == -3
    assert lib.leverage_css(ctypes.byref(good), 8, 16, 3, 0, 0, None, None, ws, 1 << 20,
                            stream) == -1  # theta
    assert lib.leverage_css(ctypes.byref(good), 8, 16, 3, 0, 9, sa, None, ws, 1 << 20,
                            stream) == -2  # prec
    assert lib.psk_probe_copy(sa, ws, 24, stream) == -1       # not a multiple of 16
    assert lib.psk_probe_copy(None, ws, 32, stream) == -1
    assert lib.psk_probe_copy(ctypes.c_void_p(0x4008), ws, 32, stream) == -1  # alignment
    assert lib.psk_probe_mfma_f64(0, sa, stream) == -1
    assert lib.psk_probe_valu_f32(10, None, stream) == -1
    assert lib.psk_probe_mfma_lowp(0, 10, sa, stream) == -2   # PSK_PREC_F64 is not a probe
    assert lib.psk_probe_mfma_lowp(1, 0, sa, stream) == -1
    assert lib.cs_hash(0, 10, 0, 0, None, None, stream) == -1
    assert lib.cs_hash(-1, 10, 5, 0, None, None, stream) == -1
    assert lib.sketch_qr(sa, 3, 5, sa, sa, ws, 1 << 20, stream) == -1
    assert lib.rownorms_sq(1.0, ctypes.byref(good), None, 3, 0.0, sa, ws, 1 << 20,
                           stream) == -1
    big = _dense(1 << 31, 5)
    assert lib.sketch_cs(ctypes.byref(big), 4, 0, sa, ws, 1 << 20, stream) == -7
    csr = _csr(10, 5, 3)
    csr.indptr = None
    assert lib.gram(1.0, ctypes.byref(csr), 0.0, sa, ws, 1 << 20, stream) == -1
    o = L.PskLsqOpts(m=2, r=8, seed=0, prec=0, max_iter=10, refine=0, check_every=1,
                     atol=1e-12, btol=1e-12)
    info = L.PskLsqInfo()
    assert lib.lsq_solve(ctypes.byref(good), sa, sa, ctypes.byref(o), ctypes.byref(info),
                         ws, 1 << 20, stream) == -1  # m < d
    o.m, o.r = 8, 4
    assert lib.lsq_solve(ctypes.byref(good), sa, sa, ctypes.byref(o), ctypes.byref(info),
                         ws, 1 << 20, stream) == -1  # r < m


def test_python_binding_reports_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_LIB", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        L.lib()


def test_server_argument_checks_before_any_device_call(lib):
    import ctypes as C
    h = C.c_void_p()
    assert lib.psk_server_create(None, C.byref(h)) == -1
    o = L.PskServerOpts(pool=None, pool_bytes=1 << 20, slots=2)
    assert lib.psk_server_create(C.byref(o), C.byref(h)) == -1      # no pool
    o = L.PskServerOpts(pool=256, pool_bytes=1 << 20, slots=0)
    assert lib.psk_server_create(C.byref(o), C.byref(h)) == -1      # slots
    o = L.PskServerOpts(pool=257, pool_bytes=1 << 20, slots=2)
    assert lib.psk_server_create(C.byref(o), C.byref(h)) == -1      # alignment
    t = C.c_int64()
    assert lib.psk_server_submit(None, None, C.byref(t)) == -1
    assert lib.psk_server_destroy(None) == -1


def test_check_planning_and_arguments(lib):
    """psk_check and the structure check every CSR call runs: a result word
    of workspace, argument errors before any device work."""
    st, c1 = _ws(L.PSK_OP_CHECK, _csr(1000, 64, 5000))
    assert st == 0 and c1 >= 4
    st, c2 = _ws(L.PSK_OP_CHECK, _dense(1000, 64))
    assert st == 0 and c2 >= 4
    # every op on CSR A reserves the word, so even the Gram of a CSR A that
    # needs no other scratch asks for some
    st, g = _ws(L.PSK_OP_GRAM, _csr(1000, 64, 5000))
    assert st == 0 and g >= 4
    assert lib.psk_check(None, 1, None, 0, None) == L.PSK_EINVAL
    # dense A without the value check: nothing to do, no device touched
    m = _dense(100, 8)
    assert lib.psk_check(ctypes.byref(m), 0, None, 0, None) == L.PSK_OK
    # a workspace too small is refused before the pass
    m = _csr(100, 8, 10)
    assert lib.psk_check(ctypes.byref(m), 0, None, 0, None) == -3
    m = _csr(100, 8, -1)
    assert lib.psk_check(ctypes.byref(m), 0, None, 0, None) == L.PSK_EINVAL
    assert L.STATUS_NAMES[L.PSK_ENONFINITE] == "PSK_ENONFINITE"


def test_checked_flag(lib):
    """PSK_MAT_CHECKED skips the per-call structure check, so a flagged CSR A
    never plans more than without it; any other flag bit or a nonzero reserved
    word is refused before any device work, for dense A as well."""
    plain = _csr(1000, 64, 5000)
    flagged = _csr(1000, 64, 5000)
    flagged.flags = L.PSK_MAT_CHECKED
    st, g0 = _ws(L.PSK_OP_GRAM, plain)
    st1, g1 = _ws(L.PSK_OP_GRAM, flagged)
    assert st == 0 and st1 == 0 and g1 <= g0
    for op in (L.PSK_OP_SKETCH_CS, L.PSK_OP_SKETCH_GCS, L.PSK_OP_ROWNORMS):
        st, a = _ws(op, plain, m=64, r=512, k=8)
        st1, b = _ws(op, flagged, m=64, r=512, k=8)
        assert st == 0 and st1 == 0 and b <= a
    # psk_check itself always runs its pass: it still needs the word
    st, c = _ws(L.PSK_OP_CHECK, flagged)
    assert st == 0 and c >= 4
    for bad in (_csr(1000, 64, 5000), _dense(1000, 64)):
        bad.flags = 2
        assert _ws(L.PSK_OP_GRAM, bad)[0] == L.PSK_EINVAL
        bad.flags, bad.reserved = 0, 1
        assert _ws(L.PSK_OP_GRAM, bad)[0] == L.PSK_EINVAL
        assert lib.psk_check(ctypes.byref(bad), 0, None, 0, None) == L.PSK_EINVAL
    d = _dense(100, 8)
    d.flags = L.PSK_MAT_CHECKED  # ignored for dense A
    assert lib.psk_check(ctypes.byref(d), 0, None, 0, None) == L.PSK_OK


def test_every_entry_point_validates_csr_first():
    """Static check of the C-ABI layer: every entry point that takes a matrix
    A runs the CSR structure check on its workspace before anything else is
    enqueued on the stream (the planning pass reserves its word too)."""
    src = open(os.path.join(ROOT, "paper_2203_02798_amd", "csrc", "abi.hip")).read()
    body = src.split('extern "C" {', 1)[1]
    funcs = re.split(r"\nint (?=\w+\()", body)
    seen = 0
    for f in funcs:
        if "check_mat(A)" not in f:
            continue
        name = f.split("(", 1)[0]
        if name == "psk_check":  # the check itself
            assert "check_operand(*A, check_values != 0, ws, as_stream(stream))" in f
            continue
        run = f.split("Arena ws = Arena::over(wsp, ws_bytes);\n", 1)
        assert len(run) == 2, name
        first = run[1].lstrip().splitlines()[0]
        assert first.startswith("if ((rc = validate_csr(*A, ws, as_stream(stream))))"), name
        plan = f.split("Arena plan;\n", 1)
        assert len(plan) == 2 and plan[1].lstrip().startswith(
            "if ((rc = validate_csr(*A, plan, nullptr)))"), name
        seen += 1
    assert seen >= 12
    serve = open(os.path.join(ROOT, "paper_2203_02798_amd", "csrc", "serve.hip")).read()
    assert "int rc = validate_csr(job->req.A, ws, st);" in serve
    assert "int rc = validate_csr(q.A, plan, nullptr);" in serve
