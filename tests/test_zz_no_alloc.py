"""sg_cgs2_noalloc (the CGS2 step whose scratch is a fixed device array) against sg_cgs2,
through the C ABI: two calls in a row, the second with a smaller input, bit-identical
coefficients and vectors (same kernels, same reduction order)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2209_14740_amd import sg  # noqa: E402


def _lib():
    L = sg.lib()
    L.sg_cgs2_noalloc.argtypes = [C.c_longlong, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.sg_cgs2_noalloc.restype = C.c_int
    return L


def _orthonormal_basis(n, nv, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, nv)) + 1j * rng.standard_normal((n, nv))
    q, _ = np.linalg.qr(a)
    return np.ascontiguousarray(q.T)   # nv vectors of length n, vector-major


def _run(fn, L, V, w):
    nv, n = V.shape
    Vd = torch.from_numpy(V).cuda()
    wd = torch.from_numpy(w.copy()).cuda()
    h = (sg.C64 * (nv + 1))()
    st = torch.cuda.current_stream().cuda_stream
    rc = getattr(L, fn)(n, nv, C.c_void_p(Vd.data_ptr()), C.c_void_p(wd.data_ptr()), C.cast(h, C.c_void_p),
                        C.c_void_p(st))
    sg.check(rc, fn)
    torch.cuda.synchronize()
    return np.array([complex(x.re, x.im) for x in h]), wd.cpu().numpy()


def test_noalloc_matches_cgs2_twice():
    L = _lib()
    L.sg_cgs2.argtypes = [C.c_longlong, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    for n, nv, seed in ((300_001, 37, 1), (4_097, 5, 2)):   # the second call is smaller
        print("noalloc case n=%d nv=%d" % (n, nv), flush=True)
        V = _orthonormal_basis(n, nv, seed)
        rng = np.random.default_rng(seed + 10)
        w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        h1, w1 = _run("sg_cgs2", L, V, w)
        h2, w2 = _run("sg_cgs2_noalloc", L, V, w)
        assert np.array_equal(h1, h2) and np.array_equal(w1, w2)
        # and what the step computes: w ⟂ V, ||w|| = 1, w h = the removed part
        assert np.max(np.abs(V.conj() @ w2)) <= 1e-13
        assert abs(np.linalg.norm(w2) - 1.0) <= 1e-13
        np.testing.assert_allclose(h2[:nv], V.conj() @ w, rtol=0, atol=1e-12 * np.linalg.norm(w))


def test_noalloc_rejects_more_than_64_vectors():
    L = _lib()
    n, nv = 1000, 65
    V = torch.zeros(nv * n, dtype=torch.complex128, device="cuda")
    w = torch.ones(n, dtype=torch.complex128, device="cuda")
    h = (sg.C64 * (nv + 1))()
    rc = L.sg_cgs2_noalloc(n, nv, C.c_void_p(V.data_ptr()), C.c_void_p(w.data_ptr()), C.cast(h, C.c_void_p),
                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1 and b"limit" in L.sg_last_error()
