"""Python binding of libpsk over PyTorch device tensors.

Every function marshals tensors into the C ABI of include/psk.h and calls it
on the current HIP stream; PyTorch only supplies device memory (outputs and
workspace) and the stream.  Names and semantics follow the C entry points.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

__all__ = [
    "CsrMatrix", "cs_hash", "sketch_cs", "sketch_gcs", "sketch_g", "gram", "rownorms_sq",
    "leverage_gram", "lsq_gram", "lsq_sketch_solve",
    "sketch_qr", "lsq_solve", "workspace_size", "version", "PskError", "Server",
]

PskError = L.PskError
_PREC = {"f64": L.PSK_PREC_F64, "bf16": L.PSK_PREC_BF16, "fp8": L.PSK_PREC_FP8}


@dataclass
class CsrMatrix:
    """CSR matrix on the device: int64 indptr (n+1), int32 indices, values
    (float64 or float32), 0-based.  ``checked`` (set by ``check(A,
    mark=True)``) passes PSK_MAT_CHECKED, so the calls skip their own
    structure check; clear it after changing indptr or indices."""
    indptr: torch.Tensor
    indices: torch.Tensor
    values: torch.Tensor
    shape: tuple
    checked: bool = False

    @property
    def device(self):
        return self.values.device

    @property
    def dtype(self):
        return self.values.dtype

    @staticmethod
    def from_scipy(m, device="cuda", dtype=None):
        dt = dtype if dtype is not None else (
            torch.float32 if m.dtype.name == "float32" else torch.float64)
        return CsrMatrix(
            torch.as_tensor(m.indptr.astype("int64"), device=device),
            torch.as_tensor(m.indices.astype("int32"), device=device),
            torch.as_tensor(m.data, device=device).to(dt),
            (int(m.shape[0]), int(m.shape[1])))


def _dtype_code(dt):
    if dt == torch.float64:
        return L.PSK_F64
    if dt == torch.float32:
        return L.PSK_F32
    raise TypeError(f"A must be float64 or float32, got {dt}")


def _mat(A):
    m = L.PskMat()
    if isinstance(A, CsrMatrix):
        if A.indptr.dtype != torch.int64 or A.indices.dtype != torch.int32:
            raise TypeError("CSR indptr must be int64 and indices int32")
        m.format = L.PSK_CSR
        m.dtype = _dtype_code(A.values.dtype)
        m.n, m.d = A.shape
        m.ld = A.shape[1]
        m.nnz = int(A.values.numel())
        m.values = A.values.data_ptr() if m.nnz else None
        m.indptr = A.indptr.data_ptr()
        m.indices = A.indices.data_ptr() if m.nnz else None
        m.flags = L.PSK_MAT_CHECKED if A.checked else 0
        return m
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise TypeError("A must be a 2-D device tensor or a CsrMatrix")
    if A.stride(1) != 1:
        raise ValueError("dense A must be row-major (unit column stride)")
    m.format = L.PSK_DENSE
    m.dtype = _dtype_code(A.dtype)
    m.n, m.d = A.shape
    m.ld = A.stride(0)
    m.nnz = 0
    m.values = A.data_ptr()
    return m


def _device(A):
    return A.device if isinstance(A, (torch.Tensor, CsrMatrix)) else torch.device("cuda")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_size(op, A, m=0, r=1, k=1, prec="f64"):
    """Minimum workspace bytes of one call (psk_workspace_size)."""
    out = ctypes.c_size_t(0)
    if isinstance(A, tuple):  # (m_rows, d) for the QR op
        mm = L.PskMat()
        mm.n, mm.d = A
        pm = mm
    else:
        pm = _mat(A)
    L.check(L.lib().psk_workspace_size(op, ctypes.byref(pm), m, r, k, _PREC[prec],
                                       ctypes.byref(out)), "psk_workspace_size")
    return int(out.value)


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def version():
    return L.lib().psk_version().decode()


def check(A, values=False, mark=False):
    """psk_check: raise PskError (PSK_EINVAL) for a malformed CSR A and, with
    values, (PSK_ENONFINITE) for a NaN or infinity among its entries.  With
    mark, a CSR A that passes gets ``A.checked = True`` (PSK_MAT_CHECKED in
    later calls)."""
    pm = _mat(A)
    dev = _device(A)
    nbytes = workspace_size(L.PSK_OP_CHECK, A)
    ws = _ws(nbytes, dev)
    L.check(L.lib().psk_check(ctypes.byref(pm), int(bool(values)), ws.data_ptr(), ws.numel(),
                              _stream(dev)), "psk_check")
    if mark and isinstance(A, CsrMatrix):
        A.checked = True


def cs_hash(count, r, seed, row0=0, device="cuda"):
    """(h int32[count], sign int8[count]) for rows row0 .. row0+count-1."""
    h = torch.empty(count, dtype=torch.int32, device=device)
    s = torch.empty(count, dtype=torch.int8, device=device)
    L.check(L.lib().cs_hash(row0, count, r, seed, h.data_ptr() if count else None,
                            s.data_ptr() if count else None,
                            _stream(torch.device(device))), "cs_hash")
    return h, s


def sketch_cs(A, r, seed, out=None):
    """S*A (r x d, dtype of A)."""
    pm = _mat(A)
    dev = _device(A)
    dt = A.dtype
    if out is None:
        out = torch.empty((r, pm.d), dtype=dt, device=dev)
    nbytes = workspace_size(L.PSK_OP_SKETCH_CS, A, r=r)
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_cs(ctypes.byref(pm), r, seed, out.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream(dev)), "sketch_cs")
    return out


def sketch_gcs(A, m, r, seed, prec="f64", out=None):
    """G*S*A (m x d, float64); m == 0 gives S*A."""
    if m == 0:
        return sketch_cs(A, r, seed, out)
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty((m, pm.d), dtype=torch.float64, device=dev)
    nbytes = workspace_size(L.PSK_OP_SKETCH_GCS, A, m=m, r=r, prec=prec)
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_gcs(ctypes.byref(pm), m, r, seed, _PREC[prec], out.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(dev)), "sketch_gcs")
    return out


def osnap_hash(count, s, r, seed, row0=0, device="cuda"):
    """(h int32[count, s], sign int8[count, s]): the rows and signs of the s
    non-zeros of columns row0 .. row0+count-1 of the OSNAP S."""
    h = torch.empty((count, s), dtype=torch.int32, device=device)
    sg = torch.empty((count, s), dtype=torch.int8, device=device)
    L.check(L.lib().osnap_hash(row0, count, s, r, seed, h.data_ptr() if count else None,
                               sg.data_ptr() if count else None,
                               _stream(torch.device(device))), "osnap_hash")
    return h, sg


def sketch_osnap(A, s, m, r, seed, prec="f64", out=None):
    """G*S*A (m x d, float64) or, with m == 0, S*A (r x d, dtype of A), S the
    OSNAP with s non-zeros per column."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        shape, dt = ((m, pm.d), torch.float64) if m > 0 else ((r, pm.d), A.dtype)
        out = torch.empty(shape, dtype=dt, device=dev)
    nbytes = workspace_size(L.PSK_OP_SKETCH_OSNAP, A, m=m, r=r, k=s, prec=prec)
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_osnap(ctypes.byref(pm), s, m, r, seed, _PREC[prec], out.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream(dev)), "sketch_osnap")
    return out


def sketch_g(A, m, seed, prec="f64", out=None):
    """G*A (m x d, float64), G the m x n Gaussian of variance 1/m."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty((m, pm.d), dtype=torch.float64, device=dev)
    nbytes = workspace_size(L.PSK_OP_SKETCH_G, A, m=m, prec=prec)
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_g(ctypes.byref(pm), m, seed, _PREC[prec], out.data_ptr(),
                             ws.data_ptr(), ws.numel(), _stream(dev)), "sketch_g")
    return out


def leverage_sketch(A, m, r, seed, t=0, prec="f64", out=None):
    """Approximate leverage scores of A (n float64): R from the sketch
    (G S A, or S A when m == 0), theta_i = ||e_i^T A R^{-1} Pi||^2 with Pi the
    d x t JL matrix (t == 0: no JL step)."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty(pm.n, dtype=torch.float64, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_LEVERAGE_SKETCH, A, m=m, r=r, k=t, prec=prec), dev)
    L.check(L.lib().leverage_sketch(ctypes.byref(pm), m, r, t, seed, _PREC[prec], out.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream(dev)), "leverage_sketch")
    return out


def css_select(A, m, r, k, seed, prec="f64"):
    """The k columns (int32 device tensor, in pivot order) that the pivoted QR
    of the sketch (G S A, or S A when m == 0) picks first."""
    pm = _mat(A)
    dev = _device(A)
    cols = torch.empty(k, dtype=torch.int32, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_CSS, A, m=m, r=r, k=k, prec=prec), dev)
    L.check(L.lib().css_select(ctypes.byref(pm), m, r, k, seed, _PREC[prec], cols.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(dev)), "css_select")
    return cols


def leverage_css(A, m, r, k, seed, prec="f64"):
    """(theta, cols): exact leverage scores of A[:, cols] (n float64) for the
    k columns css_select picks."""
    pm = _mat(A)
    dev = _device(A)
    theta = torch.empty(pm.n, dtype=torch.float64, device=dev)
    cols = torch.empty(k, dtype=torch.int32, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_LEVERAGE_CSS, A, m=m, r=r, k=k, prec=prec), dev)
    L.check(L.lib().leverage_css(ctypes.byref(pm), m, r, k, seed, _PREC[prec], theta.data_ptr(),
                                 cols.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)),
            "leverage_css")
    return theta, cols


def leverage_gram(A, out=None):
    """Exact leverage scores of A (n float64) from its Gram matrix."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty(pm.n, dtype=torch.float64, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_LEVERAGE_GRAM, A), dev)
    L.check(L.lib().leverage_gram(ctypes.byref(pm), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream(dev)), "leverage_gram")
    return out


def lsq_gram(A, b, out=None):
    """argmin ||A x - b|| (d float64) by the normal equations, B = A^T A."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty(pm.d, dtype=torch.float64, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_LSQ_GRAM, A), dev)
    L.check(L.lib().lsq_gram(ctypes.byref(pm), b.data_ptr(), out.data_ptr(), ws.data_ptr(),
                             ws.numel(), _stream(dev)), "lsq_gram")
    return out


def lsq_sketch_solve(A, b, m, r, seed, prec="f64", out=None):
    """argmin ||G S (A x - b)|| (d float64): sketch-and-solve."""
    pm = _mat(A)
    dev = _device(A)
    if out is None:
        out = torch.empty(pm.d, dtype=torch.float64, device=dev)
    ws = _ws(workspace_size(L.PSK_OP_LSQ_SKETCH, A, m=m, r=r, prec=prec), dev)
    L.check(L.lib().lsq_sketch_solve(ctypes.byref(pm), b.data_ptr(), out.data_ptr(), m, r, seed,
                                     _PREC[prec], ws.data_ptr(), ws.numel(), _stream(dev)),
            "lsq_sketch_solve")
    return out


def gram(A, alpha=1.0, beta=0.0, C=None):
    """alpha*A^T A + beta*C (d x d, dtype of A)."""
    pm = _mat(A)
    dev = _device(A)
    if C is None:
        C = torch.empty((pm.d, pm.d), dtype=A.dtype, device=dev)
        beta = 0.0
    nbytes = workspace_size(L.PSK_OP_GRAM, A)
    ws = _ws(nbytes, dev)
    L.check(L.lib().gram(alpha, ctypes.byref(pm), beta, C.data_ptr(), ws.data_ptr(),
                         ws.numel(), _stream(dev)), "gram")
    return C


def rownorms_sq(A, B, alpha=1.0, beta=0.0, x=None):
    """alpha*||e_i^T A B||^2 + beta*x_i (float64 n-vector)."""
    pm = _mat(A)
    dev = _device(A)
    B = B.contiguous()
    if B.dtype != torch.float64:
        raise TypeError("B must be float64")
    k = B.shape[1]
    if x is None:
        x = torch.empty(pm.n, dtype=torch.float64, device=dev)
        beta = 0.0
    nbytes = workspace_size(L.PSK_OP_ROWNORMS, A, k=k)
    ws = _ws(nbytes, dev)
    L.check(L.lib().rownorms_sq(alpha, ctypes.byref(pm), B.data_ptr(), k, beta,
                                x.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)),
            "rownorms_sq")
    return x


def sketch_qr(C):
    """(R, R^{-1}) of an FP64 m x d sketch (m >= d)."""
    C = C.contiguous()
    m, d = C.shape
    dev = C.device
    R = torch.empty((d, d), dtype=torch.float64, device=dev)
    Ri = torch.empty((d, d), dtype=torch.float64, device=dev)
    nbytes = workspace_size(L.PSK_OP_QR, (m, d))
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_qr(C.data_ptr(), m, d, R.data_ptr(), Ri.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream(dev)), "sketch_qr")
    return R, Ri


def sketch_qr_noalloc(C, R=None, Rinv=None):
    """(R, R^{-1}) as sketch_qr, with the library's static scratch instead of
    a workspace (no device allocation inside the call; R and Rinv may be
    passed in preallocated)."""
    C = C.contiguous()
    m, d = C.shape
    dev = C.device
    if R is None:
        R = torch.empty((d, d), dtype=torch.float64, device=dev)
    if Rinv is None:
        Rinv = torch.empty((d, d), dtype=torch.float64, device=dev)
    L.check(L.lib().sketch_qr_noalloc(C.data_ptr(), m, d, R.data_ptr(), Rinv.data_ptr(),
                                      _stream(dev)), "sketch_qr_noalloc")
    return R, Rinv


_PREC_NAME = {L.PSK_PREC_F64: "f64", L.PSK_PREC_BF16: "bf16", L.PSK_PREC_FP8: "fp8", -1: None}


def sketch_delta(Chat, C):
    """delta = ||(Chat - C) R^{-1}||_2 (R from the QR of C), both m x d FP64
    device tensors; returns a one-element FP64 device tensor."""
    Chat = Chat.contiguous()
    C = C.contiguous()
    if Chat.shape != C.shape or C.dtype != torch.float64 or Chat.dtype != torch.float64:
        raise ValueError("Chat and C must be float64 tensors of one shape")
    m, d = C.shape
    dev = C.device
    out = torch.empty(1, dtype=torch.float64, device=dev)
    nbytes = workspace_size(L.PSK_OP_DELTA, (m, d))
    ws = _ws(nbytes, dev)
    L.check(L.lib().sketch_delta(Chat.data_ptr(), C.data_ptr(), m, d, out.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream(dev)), "sketch_delta")
    return out


def lsq_solve(A, b, m=0, r=0, seed=0, prec="f64", max_iter=300, refine=1,
              check_every=8, atol=1e-14, btol=1e-14, Rinv=None, raise_on_noconv=False,
              escalate_cond=0.0, want_delta=False):
    """x = argmin ||A x - b|| by sketch-and-precondition LSQR.  With ``Rinv``
    (d x d FP64 device tensor, e.g. from sketch_qr) the preconditioner is
    reused and m, r, seed, prec are ignored.  Returns (x float64[d], info)."""
    pm = _mat(A)
    dev = _device(A)
    b = b.contiguous()
    x = torch.empty(pm.d, dtype=torch.float64, device=dev)
    if Rinv is not None:
        Rinv = Rinv.contiguous()
        if Rinv.dtype != torch.float64 or tuple(Rinv.shape) != (pm.d, pm.d):
            raise ValueError("Rinv must be a float64 d x d tensor")
    o = L.PskLsqOpts(Rinv=Rinv.data_ptr() if Rinv is not None else None, m=m, r=r,
                     seed=seed, prec=_PREC[prec], max_iter=max_iter, refine=refine,
                     check_every=check_every, atol=atol, btol=btol,
                     escalate_cond=escalate_cond, want_delta=int(bool(want_delta)))
    info = L.PskLsqInfo()
    nbytes = workspace_size(L.PSK_OP_LSQ, A, m=0 if Rinv is not None else m, r=r,
                            k=int(bool(want_delta)), prec=prec)
    ws = _ws(nbytes, dev)
    st = L.lib().lsq_solve(ctypes.byref(pm), b.data_ptr(), x.data_ptr(), ctypes.byref(o),
                           ctypes.byref(info), ws.data_ptr(), ws.numel(), _stream(dev))
    if st != L.PSK_OK and (st != -5 or raise_on_noconv):
        L.check(st, "lsq_solve")
    return x, dict(iters=info.iters, status=L.STATUS_NAMES.get(info.status, info.status),
                   resid=info.resid, ne_resid=info.ne_resid,
                   prec_used=_PREC_NAME.get(info.prec_used, info.prec_used),
                   delta_est=info.delta_est)


class Server:
    """Continuous-batching request server (psk_server_* in include/psk.h).

    ``pool_bytes`` of device memory are allocated here (torch) and handed to
    the library, which carves request workspaces out of it; ``slots``
    requests run on the device at once, each on its own HIP stream.  The
    tensors of a request are kept referenced until its result is collected
    (``wait`` / ``poll``)."""

    def __init__(self, pool_bytes, slots=4, device="cuda"):
        self.device = torch.device(device)
        self._pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        o = L.PskServerOpts(pool=self._pool.data_ptr(), pool_bytes=int(pool_bytes),
                            slots=int(slots))
        h = ctypes.c_void_p()
        L.check(L.lib().psk_server_create(ctypes.byref(o), ctypes.byref(h)),
                "psk_server_create")
        self._h = h
        self._keep = {}

    def _submit(self, op, A, b, out, opts):
        # inputs written on the current stream must be complete before a
        # worker stream reads them
        torch.cuda.current_stream(self.device).synchronize()
        q = L.PskRequest(op=op, A=_mat(A), b=b.data_ptr() if b is not None else None,
                         out=out.data_ptr(), opts=opts)
        t = ctypes.c_int64()
        L.check(L.lib().psk_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)),
                "psk_server_submit")
        self._keep[t.value] = (A, b, out)
        return t.value

    def submit_lsq(self, A, b, m, r, seed=0, prec="f64", max_iter=300, refine=1,
                   check_every=8, atol=1e-14, btol=1e-14, escalate_cond=0.0,
                   want_delta=False):
        """Queue x = argmin ||A x - b||; returns (ticket, x) with x filled on
        completion."""
        pm = _mat(A)
        x = torch.empty(pm.d, dtype=torch.float64, device=self.device)
        o = L.PskLsqOpts(Rinv=None, m=m, r=r, seed=seed, prec=_PREC[prec],
                         max_iter=max_iter, refine=refine, check_every=check_every,
                         atol=atol, btol=btol, escalate_cond=escalate_cond,
                         want_delta=int(bool(want_delta)))
        return self._submit(L.PSK_REQ_LSQ, A, b.contiguous(), x, o), x

    def submit_leverage(self, A, m, r, seed=0, prec="f64"):
        """Queue sketched leverage scores; returns (ticket, theta)."""
        pm = _mat(A)
        th = torch.empty(pm.n, dtype=torch.float64, device=self.device)
        o = L.PskLsqOpts(Rinv=None, m=m, r=r, seed=seed, prec=_PREC[prec], max_iter=1,
                         refine=0, check_every=1, atol=0.0, btol=0.0)
        return self._submit(L.PSK_REQ_LEVERAGE, A, None, th, o), th

    @staticmethod
    def _result(res):
        return dict(status=L.STATUS_NAMES.get(res.status, res.status), iters=res.iters,
                    resid=res.resid, ne_resid=res.ne_resid, t_submit=res.t_submit,
                    t_start=res.t_start, t_end=res.t_end,
                    prec_used=_PREC_NAME.get(res.prec_used, res.prec_used),
                    delta_est=res.delta_est)

    def wait(self, ticket):
        res = L.PskResult()
        L.check(L.lib().psk_server_wait(self._h, ticket, ctypes.byref(res)),
                "psk_server_wait")
        self._keep.pop(ticket, None)
        return self._result(res)

    def poll(self, ticket):
        """The result dict if finished, else None."""
        res = L.PskResult()
        st = L.lib().psk_server_poll(self._h, ticket, ctypes.byref(res))
        if st == L.PSK_PENDING:
            return None
        L.check(st, "psk_server_poll")
        self._keep.pop(ticket, None)
        return self._result(res)

    def stats(self):
        s = L.PskServerStats()
        L.check(L.lib().psk_server_stats(self._h, ctypes.byref(s)), "psk_server_stats")
        return {k: getattr(s, k) for k, _ in L.PskServerStats._fields_}

    def close(self):
        if self._h is not None:
            L.check(L.lib().psk_server_destroy(self._h), "psk_server_destroy")
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def measure_ceilings(device="cuda:0", copy_bytes=1 << 30, reps=3):
    """Rates this device sustains (the ceiling probes, each timed with events
    on the launch stream, best of ``reps``): HBM GB/s of a plain copy (bytes
    read + written), FP64 / BF16 / FP8 matrix TFLOP/s, VALU tera
    lane-operations/s."""
    dev = torch.device(device)
    st = _stream(dev)
    stream = torch.cuda.current_stream(dev)
    src = torch.ones(copy_bytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    outd = torch.empty(L.PSK_PROBE_BLOCKS * 256, dtype=torch.float64, device=dev)
    outf = torch.empty(L.PSK_PROBE_BLOCKS * 256, dtype=torch.float32, device=dev)

    def best(launch):
        launch()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts)

    t = best(lambda: L.check(L.lib().psk_probe_copy(src.data_ptr(), dst.data_ptr(), copy_bytes,
                                                    st), "psk_probe_copy"))
    hbm = 2.0 * copy_bytes / t / 1e9
    it_m = 1000
    t = best(lambda: L.check(L.lib().psk_probe_mfma_f64(it_m, outd.data_ptr(), st),
                             "psk_probe_mfma_f64"))
    mfma = L.PSK_PROBE_BLOCKS * 4 * it_m * 8 * 2048.0 / t / 1e12
    it_b = 100
    t = best(lambda: L.check(L.lib().psk_probe_mfma_lowp(L.PSK_PREC_BF16, it_b, outf.data_ptr(),
                                                         st), "psk_probe_mfma_lowp"))
    bf16 = L.PSK_PROBE_BLOCKS * 4 * it_b * 8 * 16384.0 / t / 1e12
    it_8 = 50
    t = best(lambda: L.check(L.lib().psk_probe_mfma_lowp(L.PSK_PREC_FP8, it_8, outf.data_ptr(),
                                                         st), "psk_probe_mfma_lowp"))
    fp8 = L.PSK_PROBE_BLOCKS * 4 * it_8 * 8 * 65536.0 / t / 1e12
    it_v = 20000
    t = best(lambda: L.check(L.lib().psk_probe_valu_f32(it_v, outf.data_ptr(), st),
                             "psk_probe_valu_f32"))
    valu = L.PSK_PROBE_BLOCKS * 256 * it_v * 8.0 / t / 1e12
    return {"hbm_copy_GBs": hbm, "fp64_mfma_TFs": mfma, "bf16_mfma_TFs": bf16,
            "fp8_mfma_TFs": fp8, "valu_Tops": valu}


class kernel_timing:
    """Context manager that enables the library's event brackets around its
    main kernels (only those named in ``only``, if given); ``stats()``
    returns {name: (total_ms, launches)}."""

    def __init__(self, only=None):
        self.only = ",".join(only).encode() if only else None

    def __enter__(self):
        L.lib().psk_timing_reset()
        L.lib().psk_timing_only(self.only)
        L.lib().psk_timing_enable(1)
        return self

    def __exit__(self, *exc):
        L.lib().psk_timing_enable(0)
        L.lib().psk_timing_only(None)
        return False

    @staticmethod
    def stats():
        names = L.lib().psk_timing_names().decode()
        out = {}
        for nm in filter(None, names.split(",")):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_int64(0)
            L.check(L.lib().psk_timing_collect(nm.encode(), ctypes.byref(ms),
                                               ctypes.byref(n)), "psk_timing_collect")
            out[nm] = (ms.value, n.value)
        return out
