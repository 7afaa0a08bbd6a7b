"""The allocation-free backward (pros_lpcost_bwd_noalloc) against the
workspace backward (pros_lpcost_bwd) through the C ABI: same kernels, so
every output is bit-identical; two calls in a row on the library's fixed
scratch, the second with a smaller problem, and the size limit refused
before any launch."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu


def _inputs(m, k, B, seed, weighted):
    import torch
    rng = np.random.default_rng([m, k, B, seed])
    U = np.linalg.qr(rng.standard_normal((m, k)))[0]
    Y = 0.05 * rng.standard_normal((B, k))
    X = Y @ U.T + 0.01 * rng.standard_normal((B, m))
    hit = rng.random((B, m)) < 0.1
    X[hit] = rng.random(hit.sum())
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    w = t(np.where(rng.random(m) < 0.2, 5e-5, 1.0)) if weighted else None
    g = t(rng.standard_normal(B))
    return t(U), t(Y), t(X), w, t([1e-3]), g


def _outputs(m, k, B):
    import torch
    z = lambda *s: torch.full(s, float("nan"), dtype=torch.float32, device="cuda")
    return z(B, m), z(m, k), z(B, k), z(1)


def _call(L, lib, noalloc, ins, outs, m, k, B, cost, p):
    import torch
    U, Y, X, w, mu, g = ins
    dX, dU, dY, dmu = outs
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        st = lib.pros_lpcost_bwd_noalloc(ptr(U), ptr(Y), ptr(X), ptr(w), ptr(mu), m, k, B, cost, p, ptr(g),
                                         ptr(dX), ptr(dU), ptr(dY), ptr(dmu), sp)
    else:
        nws = lib.pros_lpcost_workspace_size(m, k, B)
        ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
        st = lib.pros_lpcost_bwd(ptr(U), ptr(Y), ptr(X), ptr(w), ptr(mu), m, k, B, cost, p, ptr(g),
                                 ptr(dX), ptr(dU), ptr(dY), ptr(dmu), ptr(ws), nws, sp)
    L.check(st)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in outs]


@pytest.mark.parametrize("cost,p", [(0, 0.25), (1, 0.25)])
def test_noalloc_backward_equals_workspace_backward(cost, p):
    from paper_1302_2073_amd import _lib as L
    lib = L.lib()
    # full differentiation workload, then a smaller ragged one on the same scratch
    for (m, k, B, weighted) in ((230400, 10, 32, False), (3001, 7, 5, True)):
        say(f"noalloc backward m={m} k={k} B={B} cost={cost} weighted={weighted}")
        ins = _inputs(m, k, B, 1, weighted)
        ref = _call(L, lib, False, ins, _outputs(m, k, B), m, k, B, cost, p)
        got = _call(L, lib, True, ins, _outputs(m, k, B), m, k, B, cost, p)
        for name, a, b in zip(("dX", "dU", "dY", "dmu"), got, ref):
            assert np.all(np.isfinite(a)), name
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), name


def test_noalloc_refuses_problems_beyond_the_scratch():
    import torch
    from paper_1302_2073_amd import _lib as L
    lib = L.lib()
    m, k, B = 4_000_000, 16, 64
    assert lib.pros_lpcost_workspace_size(m, k, B) > L.PROS_LPCOST_SCRATCH_BYTES
    one = torch.zeros(1, dtype=torch.float32, device="cuda")
    p = C.c_void_p(one.data_ptr())
    st = lib.pros_lpcost_bwd_noalloc(p, p, p, None, p, m, k, B, 0, 0.25, p, None, None, None, None,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.PROS_EINVAL
    assert "scratch" in L.last_error()
