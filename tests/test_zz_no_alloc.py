"""sketch_qr_noalloc (no device allocation: the library's static scratch)
against sketch_qr (a caller workspace) through the C ABI: two calls in a row,
the second smaller, each bit for bit equal to the workspace form; a shape
beyond the static scratch is refused."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2203_02798_amd import api as a
    return a


def _sketch(m, d, cond, seed):
    c, _, _ = synth.lsq_problem(m, d, cond, seed=seed, noise=0.0)
    return torch.from_numpy(c).cuda()


@pytest.mark.gpu
def test_sketch_qr_noalloc_matches_workspace_form(api):
    L = api.L
    for (m, d, cond, seed) in ((2000, 500, 1e6, 1), (300, 40, 1e2, 2)):
        print(f"sketch_qr_noalloc m={m} d={d} cond={cond:g}", flush=True)
        c = _sketch(m, d, cond, seed)
        r_ws, ri_ws = api.sketch_qr(c)
        r = torch.full((d, d), float("nan"), dtype=torch.float64, device="cuda")
        ri = torch.full((d, d), float("nan"), dtype=torch.float64, device="cuda")
        st = L.lib().sketch_qr_noalloc(c.data_ptr(), m, d, r.data_ptr(), ri.data_ptr(),
                                       api._stream(c.device))
        assert st == L.PSK_OK, L.lib().psk_last_error()
        torch.cuda.synchronize()
        assert torch.equal(r, r_ws) and torch.equal(ri, ri_ws)
        # and the factor is right: R^T R = C^T C
        rh, ch = r.cpu().numpy(), c.cpu().numpy()
        assert np.linalg.norm(rh.T @ rh - ch.T @ ch) / np.linalg.norm(ch.T @ ch) <= 1e-13


@pytest.mark.gpu
def test_sketch_qr_noalloc_refuses_oversize(api):
    L = api.L
    m, d = 20000, 2000  # about 2 m d + 11 d^2 doubles: far beyond 64 MiB
    st = L.lib().sketch_qr_noalloc(ctypes.c_void_p(1), m, d, ctypes.c_void_p(1),
                                   ctypes.c_void_p(1), None)
    assert st == -7
    assert b"PSK_NOALLOC_SCRATCH_BYTES" in L.lib().psk_last_error()
