"""Calls on two streams at once: the Gram matrix on a second stream beside
the sketch, its QR and the row norms on the first (the order the headline
step uses) give the same bits as the same calls one after another, dense
and CSR.  Every call's workspace comes from the caching allocator on the
stream the call runs on."""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def api():
    from paper_2203_02798_amd import api as a
    return a


def _serial(api, A, m, r, seed):
    C = api.sketch_gcs(A, m, r, seed)
    G = api.gram(A)
    _, Ri = api.sketch_qr(C)
    th = api.rownorms_sq(A, Ri)
    return C, G, Ri, th


def _two_streams(api, A, m, r, seed, side):
    main = torch.cuda.current_stream()
    side.wait_stream(main)
    with torch.cuda.stream(side):
        G = api.gram(A)
    C = api.sketch_gcs(A, m, r, seed)
    _, Ri = api.sketch_qr(C)
    th = api.rownorms_sq(A, Ri)
    main.wait_stream(side)
    G.record_stream(main)
    return C, G, Ri, th


@pytest.mark.parametrize("kind", ["dense32", "csr"])
def test_gram_beside_sketch_same_bits(api, kind):
    if kind == "dense32":
        A = synth.dense_coherent_torch(300_000, 256, seed=5)
        m, r = 512, 8192
    else:
        a = synth.csr_uniform(400_000, 300, 5e-3, seed=5)
        A = api.CsrMatrix.from_scipy(a, device="cuda:0")
        m, r = 600, 40_000
    side = torch.cuda.Stream()  # default priority
    want = _serial(api, A, m, r, 7)
    torch.cuda.synchronize()
    for _ in range(3):
        got = _two_streams(api, A, m, r, 7, side)
        torch.cuda.synchronize()
        for w, g in zip(want, got):
            assert torch.equal(w, g)
