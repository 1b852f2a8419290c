"""ctypes wrapper of the C oracle (jacobi_oracle.c) -- test infrastructure only.

Each function cites the passage of Demmel, Luo, Schneider, Wang, "Parallel
Jacobi, Part Two" (arXiv 2608.28952) that it follows; see jacobi_oracle.c.
Matrices cross the boundary as column-major (Fortran-order) float64 arrays.
"""
import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.OUT):
            build_oracle.build()
        L = ctypes.CDLL(build_oracle.OUT)
        L.ora_eig.restype = ctypes.c_int
        L.ora_eig.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp,
                              ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_longlong, _dp, _ip,
                              ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        L.ora_svd.restype = ctypes.c_int
        L.ora_svd.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int,
                              _dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              _ip, ctypes.POINTER(ctypes.c_longlong)]
        L.ora_gram.restype = None
        L.ora_gram.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int, _ip, _dp]
        L.ora_qr.restype = ctypes.c_int
        L.ora_qr.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int]
        L.ora_antidiag_list.restype = ctypes.c_int
        L.ora_antidiag_list.argtypes = [ctypes.c_int, _ip, _ip]
        L.ora_rr_list.restype = ctypes.c_int
        L.ora_rr_list.argtypes = [ctypes.c_int, _ip, _ip]
        L.ora_block_step.restype = ctypes.c_int
        L.ora_block_step.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _ip, _dp, _dp]
        L.ora_offnorm.restype = ctypes.c_double
        L.ora_offnorm.argtypes = [ctypes.c_int, _dp, ctypes.c_int]
        L.ora_check_offnorm.restype = ctypes.c_double
        L.ora_check_offnorm.argtypes = [ctypes.c_int, _dp, ctypes.c_int]
        L.ora_check_eig.restype = None
        L.ora_check_eig.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
        L.ora_check_eig_sampled.restype = None
        L.ora_check_eig_sampled.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                            ctypes.c_int, _ip, _dp]
        L.ora_check_svd.restype = None
        L.ora_check_svd.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp,
                                    ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.ora_cayley.restype = ctypes.c_int
        L.ora_lupp_cols.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _ip]
        L.ora_cayley.argtypes = [ctypes.c_int, _dp, _dp]
        L.ora_cayley_inverse.restype = ctypes.c_int
        L.ora_cayley_inverse.argtypes = [ctypes.c_int, _dp, _dp]
        _lib = L
    return _lib


def _f64(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


class OracleResult(dict):
    __getattr__ = dict.__getitem__


def eig(A, tol=1e-14, max_sweeps=50, order=1, Q0=None, want_vectors=True, nthreads=1,
        check_rotations=False, max_rotations=0, relative=False):
    """Scalar cyclic Jacobi (Alg. 1 with b = 1).  Returns W ascending, Q, sweeps,
    rotations, status and (optionally) the largest relative deviation from the
    per-rotation identity off^2 -= 2 a_pq^2 (§1).  relative=True: rotate only
    when |a_pq| > tol sqrt(|a_pp a_qq|), stop after a sweep without rotations
    (the Demmel-Veselic threshold)."""
    A = _f64(A)
    n = A.shape[0]
    W = np.zeros(n)
    Q = np.zeros((n, n), order="F") if want_vectors else None
    Q0a = _f64(Q0) if Q0 is not None else None
    sw = ctypes.c_int(0)
    nr = ctypes.c_longlong(0)
    chk = ctypes.c_double(0.0)
    rc = lib().ora_eig(n, _p(A), max(n, 1), _p(W), _p(Q), max(n, 1), _p(Q0a), max(n, 1),
                       tol, max_sweeps, order, nthreads, max_rotations,
                       ctypes.byref(chk) if check_rotations else None, ctypes.byref(sw),
                       ctypes.byref(nr), 1 if relative else 0)
    return OracleResult(W=W, Q=Q, sweeps=sw.value, rotations=nr.value, status=rc,
                        rot_identity=chk.value)


def svd(G, tol=None, max_sweeps=60, order=1, nthreads=1):
    """One-sided Jacobi SVD (Alg. 6 with b = 1, Hestenes).  Returns S
    descending, U (m x n), V (n x n), sweeps, status.  nthreads > 1 (with the
    round-robin order) rotates the disjoint pairs of a round in parallel,
    with the same result."""
    G = _f64(G)
    m, n = G.shape
    if tol is None:
        tol = np.sqrt(m) * np.finfo(np.float64).eps
    S = np.zeros(n)
    U = np.zeros((m, n), order="F")
    V = np.zeros((n, n), order="F")
    sw = ctypes.c_int(0)
    nr = ctypes.c_longlong(0)
    rc = lib().ora_svd(m, n, _p(G), max(m, 1), _p(S), _p(U), max(m, 1), _p(V), max(n, 1),
                       tol, max_sweeps, order, nthreads, ctypes.byref(sw), ctypes.byref(nr))
    return OracleResult(S=S, U=U, V=V, sweeps=sw.value, rotations=nr.value, status=rc)


def gram(G, cols_a, cols_b):
    """G(:, cols_a)^T G(:, cols_b) summed in long double (eq. SVD_subproblem, §6)."""
    G = _f64(G)
    m = G.shape[0]
    ca = np.ascontiguousarray(cols_a, dtype=np.int32)
    cb = np.ascontiguousarray(cols_b, dtype=np.int32)
    out = np.zeros((len(ca), len(cb)), order="F")
    lib().ora_gram(m, _p(G), max(m, 1), len(ca), ca.ctypes.data_as(_ip), len(cb), cb.ctypes.data_as(_ip), _p(out))
    return out


def qr(G, want_q=True):
    """Reduced QR G = Q R (m >= n) by Householder reflections in long double,
    diag(R) >= 0 (the preprocessing of the one-sided SVD, §6)."""
    G = _f64(G)
    m, n = G.shape
    Q = np.zeros((m, n), order="F") if want_q else None
    R = np.zeros((n, n), order="F")
    rc = lib().ora_qr(m, n, _p(G), max(m, 1), _p(Q), max(m, 1), _p(R), max(n, 1))
    assert rc == 0, rc
    return Q, R


def antidiag_list(P):
    """Alg. 3: list of P groups of 0-based pairs (I, J)."""
    pairs = np.zeros(max(P * (P - 1), 2), dtype=np.int32)
    sizes = np.zeros(max(P, 1), dtype=np.int32)
    lib().ora_antidiag_list(P, pairs.ctypes.data_as(_ip), sizes.ctypes.data_as(_ip))
    out, base = [], 0
    for K in range(P):
        k = int(sizes[K])
        out.append([(int(pairs[2 * (base + i)]), int(pairs[2 * (base + i) + 1])) for i in range(k)])
        base += k
    return out


def rr_list(N):
    """Round-robin rounds (list of lists of 0-based pairs)."""
    pairs = np.zeros(max(N * (N - 1), 2), dtype=np.int32)
    sizes = np.zeros(max(N + 1, 1), dtype=np.int32)
    R = lib().ora_rr_list(N, pairs.ctypes.data_as(_ip), sizes.ctypes.data_as(_ip))
    out, base = [], 0
    for K in range(R):
        k = int(sizes[K])
        out.append([(int(pairs[2 * (base + i)]), int(pairs[2 * (base + i) + 1])) for i in range(k)])
        base += k
    return out


def block_step(A, Q, b, pairs, Vhat, Dhat=None):
    """One parallel step of Alg. 2 in long double; returns (A_new, Q_new)."""
    A = _f64(A).copy(order="F")
    Q = _f64(Q).copy(order="F") if Q is not None else None
    n = A.shape[0]
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    Vh = np.ascontiguousarray(np.stack([np.asfortranarray(v).reshape(-1, order="F") for v in Vhat]))
    Dh = None
    if Dhat is not None:
        Dh = np.ascontiguousarray(np.stack([np.asfortranarray(d).reshape(-1, order="F") for d in Dhat]))
    rc = lib().ora_block_step(n, b, _p(A), _p(Q), len(pairs), pr.ctypes.data_as(_ip),
                              Vh.ctypes.data_as(_dp), Dh.ctypes.data_as(_dp) if Dh is not None else None)
    assert rc == 0, rc
    return A, Q


def offnorm(A):
    A = _f64(A)
    return lib().ora_offnorm(A.shape[0], _p(A), max(A.shape[0], 1))


def check_offnorm(A):
    A = _f64(A)
    return lib().ora_check_offnorm(A.shape[0], _p(A), max(A.shape[0], 1))


def check_eig(A, W, Q):
    """Long double: (||A - Q diag(W) Q^T||_F/||A||_F, ||Q^T Q - I||_F,
    trace(A) - sum W, (||A||_F^2 - sum W^2)/||A||_F^2)."""
    A = _f64(A)
    Q = _f64(Q)
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.zeros(4)
    n = A.shape[0]
    lib().ora_check_eig(n, _p(A), max(n, 1), _p(W), _p(Q), max(n, 1), _p(out))
    return out


def check_eig_sampled(A, W, Q, cols):
    A = _f64(A)
    Q = _f64(Q)
    W = np.ascontiguousarray(W, dtype=np.float64)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.zeros(2)
    n = A.shape[0]
    lib().ora_check_eig_sampled(n, _p(A), n, _p(W), _p(Q), n, len(c), c.ctypes.data_as(_ip), _p(out))
    return out


def check_svd(G, S, U, V):
    """Long double: (||G - U S V^T||_F/||G||_F, ||V^T V - I||_F, ||U^T U - I||_F)."""
    G = _f64(G)
    U = _f64(U)
    V = _f64(V)
    S = np.ascontiguousarray(S, dtype=np.float64)
    m, n = G.shape
    out = np.zeros(3)
    lib().ora_check_svd(m, n, _p(G), m, _p(S), _p(U), m, _p(V), n, _p(out))
    return out


def lupp_cols(M):
    """Column permutation of the pivoting step (§2.1): LU with partial
    pivoting on M^T for M rows x cols (rows <= cols).  Returns perm (cols
    ints): column j of M P is column perm[j] of M."""
    M = _f64(M)
    rows, cols = M.shape
    perm = np.zeros(cols, dtype=np.int32)
    rc = lib().ora_lupp_cols(rows, cols, _p(M), max(rows, 1), perm.ctypes.data_as(_ip))
    if rc != 0:
        raise ValueError(f"ora_lupp_cols: {rc}")
    return perm


def cayley(S):
    """W = (I - S)^{-1} (I + S), long double Gaussian elimination."""
    S = _f64(S)
    n = S.shape[0]
    W = np.zeros((n, n), order="F")
    rc = lib().ora_cayley(n, _p(S), _p(W))
    assert rc == 0
    return W


def cayley_inverse(W):
    """S = (W - I)(W + I)^{-1}."""
    W = _f64(W)
    n = W.shape[0]
    S = np.zeros((n, n), order="F")
    rc = lib().ora_cayley_inverse(n, _p(W), _p(S))
    assert rc == 0
    return S


def check_svd_sampled(G, S, U, V, cols):
    """Long double, sampled columns: (max ||G v_c - s_c u_c|| / ||G||_F,
    max |V^T V - I| entry, max |U^T U - I| entry over the samples)."""
    L = lib()
    if not hasattr(L, "_svd_sampled_set"):
        L.ora_check_svd_sampled.restype = None
        L.ora_check_svd_sampled.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                            _dp, ctypes.c_int, ctypes.c_int, _ip, _dp]
        L._svd_sampled_set = True
    G = _f64(G)
    U = _f64(U)
    V = _f64(V)
    S = np.ascontiguousarray(S, dtype=np.float64)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    m, n = G.shape
    out = np.zeros(3)
    L.ora_check_svd_sampled(m, n, _p(G), m, _p(S), _p(U), m, _p(V), n, len(c), c.ctypes.data_as(_ip), _p(out))
    return out
