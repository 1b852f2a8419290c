"""jacobi_eig_noalloc (workspace in the library's static device array)
against jacobi_eig with a caller workspace, through the C-ABI: two calls in a
row, the second on a smaller matrix, each compared with the existing entry
point's result (eigenvalues within 1e-12 max|lambda|, and the long-double
residual and orthogonality of both within 1e-12)."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_28952_amd import inputs

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2608_28952_amd import jacobi as jx
    L = jx.lib()
    L.jacobi_eig_noalloc.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_char, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(jx.Opts), ctypes.POINTER(jx.Info), ctypes.c_void_p]
    L.jacobi_eig_noalloc_max_bytes.restype = ctypes.c_size_t
    return jx, L


def _solve(jx, L, A_np, noalloc, **kw):
    import torch
    n = A_np.shape[0]
    o = jx.opts_default(**kw)
    A = torch.from_numpy(np.asfortranarray(A_np).reshape(-1, order="F").copy()).cuda()  # column-major
    W = torch.empty(n, dtype=torch.float64, device="cuda")
    Q = torch.empty(n * n, dtype=torch.float64, device="cuda")
    info = jx.Info()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = L.jacobi_eig_noalloc(n, A.data_ptr(), n, b"U", W.data_ptr(), Q.data_ptr(), n, None, n,
                                  ctypes.byref(o), ctypes.byref(info), s)
    else:
        work = torch.empty(L.jacobi_eig_workspace(n, ctypes.byref(o)), dtype=torch.uint8, device="cuda")
        rc = L.jacobi_eig(n, A.data_ptr(), n, b"U", W.data_ptr(), Q.data_ptr(), n, None, n, work.data_ptr(),
                          work.numel(), ctypes.byref(o), ctypes.byref(info), s)
    torch.cuda.synchronize()
    return rc, W.cpu().numpy(), Q.cpu().numpy().reshape((n, n), order="F"), info.as_dict()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_point(prec):
    jx, L = _lib()
    kw = {"precision": jx.PREC_MIXED_FP32 if prec == "mixed" else jx.PREC_FP64}
    for n, seed in ((1000, 31), (300, 32)):  # second call smaller: stale contents must not matter
        print(f"noalloc n={n} prec={prec}", flush=True)
        A, _ = inputs.eig_uniform(n, seed)
        rc1, W1, Q1, i1 = _solve(jx, L, A, True, **kw)
        rc0, W0, Q0, i0 = _solve(jx, L, A, False, **kw)
        assert rc1 == 0 and rc0 == 0, (rc1, rc0, jx.last_error())
        scale = np.max(np.abs(W0))
        assert np.max(np.abs(W1 - W0)) <= 1e-12 * scale
        for W, Q in ((W1, Q1), (W0, Q0)):
            res, orth, _, _ = O.check_eig(A, W, Q)
            assert res <= 1e-12 and orth <= 1e-12, (res, orth)
        print(f"  sweeps {i1['sweeps']} / {i0['sweeps']}, bitwise equal W: {np.array_equal(W1, W0)}", flush=True)


def test_noalloc_rejects_orders_beyond_the_array():
    import torch
    jx, L = _lib()
    cap = L.jacobi_eig_noalloc_max_bytes()
    n = 4096
    o = jx.opts_default()
    assert L.jacobi_eig_workspace(n, ctypes.byref(o)) > cap
    dummy = torch.empty(8, dtype=torch.float64, device="cuda")
    info = jx.Info()
    rc = L.jacobi_eig_noalloc(n, dummy.data_ptr(), n, b"U", dummy.data_ptr(), dummy.data_ptr(), n, None, n,
                              ctypes.byref(o), ctypes.byref(info), None)
    assert rc == -1 and info.status == -1
    assert "static scratch array" in jx.last_error()
