"""Thin ctypes binding of libjacobi.so (include/jacobi.h).

Argument marshalling only: every step of the solvers runs in the library's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.  If
the built library is missing, every call raises; there is no fallback.

Layout: the library is column-major.  A torch tensor is row-major, so a
row-major n x n buffer read as column-major is the transpose; the wrappers
below handle that (symmetric inputs flip `uplo`; outputs are returned as
transposed views so that ``Q[:, j]`` is eigenvector j).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libjacobi.so")

_lib = None

ORDER_ROUND_ROBIN = 0
ORDER_ANTIDIAG = 1
ORDER_ROUND_ROBIN_SORTED = 2
PREC_FP64 = 0
PREC_MIXED_FP32 = 1
PREC_MIXED_BF16 = 2
F32 = 0
F64 = 1


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int), ("block", ctypes.c_int),
                ("ordering", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_max_sweeps", ctypes.c_int), ("refine", ctypes.c_int), ("sort", ctypes.c_int),
                ("want_vectors", ctypes.c_int), ("threshold", ctypes.c_int), ("precondition", ctypes.c_int),
                ("pivot", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sweeps", ctypes.c_int), ("sweeps_by_prec", ctypes.c_int * 3),
                ("fallback_used", ctypes.c_int), ("off_rel", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "sweeps": self.sweeps, "sweeps_by_prec": list(self.sweeps_by_prec),
                "fallback_used": self.fallback_used, "off_rel": self.off_rel, "seconds": self.seconds}


def _info_dtype():
    """numpy structured dtype with the layout of jacobi_info (Info)."""
    import numpy as np
    dt = np.dtype([("status", "i4"), ("sweeps", "i4"), ("sweeps_by_prec", "i4", (3,)), ("fallback_used", "i4"),
                   ("off_rel", "f8"), ("seconds", "f8")], align=True)
    assert dt.itemsize == ctypes.sizeof(Info)
    return dt


def _info_dicts(a, count):
    """as_dict() of the first `count` entries of an Info array held as a
    numpy structured array, read column by column (per-field ctypes access
    costs about 2 us per matrix on large batches)."""
    if count <= 0:
        return []
    a = a[:count]
    st, sw, sp = a["status"].tolist(), a["sweeps"].tolist(), a["sweeps_by_prec"].tolist()
    fb, off, sec = a["fallback_used"].tolist(), a["off_rel"].tolist(), a["seconds"].tolist()
    return [{"status": st[k], "sweeps": sw[k], "sweeps_by_prec": sp[k], "fallback_used": fb[k],
             "off_rel": off[k], "seconds": sec[k]} for k in range(count)]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    """Load libjacobi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libjacobi.so not built ({LIB_PATH}); run python -m paper_2608_28952_amd.build")
        # PyTorch first: its HIP runtime is then the one the library binds to
        # (loaded the other way round, the process holds two HIP runtimes and
        # the library's sees no device)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.jacobi_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.jacobi_last_error.restype = ctypes.c_char_p
        L.jacobi_eig_workspace.restype = ctypes.c_size_t
        L.jacobi_eig_workspace.argtypes = [ctypes.c_int, ctypes.POINTER(Opts)]
        L.jacobi_svd_workspace.restype = ctypes.c_size_t
        L.jacobi_svd_workspace.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Opts)]
        L.jacobi_eig_batched_workspace.restype = ctypes.c_size_t
        L.jacobi_eig_batched_workspace.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.POINTER(Opts)]
        L.jacobi_eig.argtypes = [ctypes.c_int, _vp, ctypes.c_int, ctypes.c_char, _vp, _vp, ctypes.c_int, _vp,
                                 ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(Opts), ctypes.POINTER(Info), _vp]
        L.jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp,
                                 ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(Opts), ctypes.POINTER(Info), _vp]
        L.jacobi_eig_batched.argtypes = [ctypes.c_int, _ip, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, _vp, _vp,
                                         _vp, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(Opts),
                                         ctypes.POINTER(Info), _vp]
        L.jacobi_schedule.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _ip]
        L.jacobi_batched_tuning.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _ip]
        L.jacobi_batched_graph_stats.argtypes = [_ip, _ip]
        L.jacobi_batched_autotune.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_char_p]
        L.jws_param_count.restype = ctypes.c_size_t
        L.jws_param_count.argtypes = []
        L.jws_acts_bytes.restype = ctypes.c_size_t
        L.jws_acts_bytes.argtypes = [ctypes.c_int]
        L.jws_mlp_forward.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
        L.jws_mlp_backward.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
        L.jws_mse.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
        L.jws_adam_step.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_int, _vp]
        L.jws_to_bf16.argtypes = [ctypes.c_size_t, _vp, _vp, _vp]
        L.jws_skew_from_coords.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
        L.jws_cayley_batched.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.jws_family_matrices.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
        L.jws_canonical_targets.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_double, _vp]
        L.jws_column_stats_work.restype = ctypes.c_size_t
        L.jws_column_stats_work.argtypes = [ctypes.c_int, ctypes.c_int]
        L.jws_column_stats.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_float, _vp, _vp,
                                       _vp, _vp]
        L.jws_gather_standardize.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                             _vp, _vp]
        L.jacobi_init.argtypes = []
        L.jacobi_subproblem_solve.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.jacobi_qr.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int,
                                _vp]
        L.jacobi_gram_blocks.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                                         _ip, ctypes.c_int, _vp, _vp]
        L.jacobi_block_step.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _ip, _vp, _vp, _vp]
        L.jacobi_block_step32.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _ip, _vp, _vp, _vp]
        L.jacobi_pivot_step.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _ip, _vp, _vp, _vp]
        _lib = L
    return _lib


def last_error():
    return lib().jacobi_last_error().decode()


def opts_default(**kw):
    o = Opts()
    lib().jacobi_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class JacobiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jacobi error {code}: {msg}")
        self.code = code


def _check(rc, allow=(0,)):
    if rc not in allow:
        raise JacobiError(rc, last_error())
    return rc


def _colmajor_view(t):
    """(ptr tensor, ld) for reading t (m x n) as column-major, copying if needed."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    if t.stride(0) == 1 and t.stride(1) >= max(t.shape[0], 1):
        return t, t.stride(1)
    c = t.t().contiguous().t()
    return c, max(c.shape[0], 1)


def jacobi_eig(A, uplo="U", Q0=None, opts=None, work=None, check=True):
    """Symmetric eigendecomposition of the float64 CUDA tensor A (n x n).

    Returns (W, Q, info) with W ascending and Q[:, j] the eigenvector of W[j]
    (Q is None when opts.want_vectors == 0).  `uplo` names the valid triangle
    of A in the usual (row, column) indexing.  With check=True a non-zero
    status raises; otherwise it is returned in info["status"]."""
    import torch
    o = opts if opts is not None else opts_default()
    n = A.shape[0]
    if A.shape != (n, n) or A.dtype != torch.float64 or not A.is_cuda:
        raise ValueError("A must be a square float64 CUDA tensor")
    if A.is_contiguous():  # row-major buffer = A^T column-major; the valid triangle flips
        Ab, lda, ul = A, max(n, 1), {"U": b"L", "L": b"U"}[uplo.upper()]
    else:
        Ab, lda = _colmajor_view(A)
        ul = uplo.upper().encode()
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Qt = torch.empty((n, n), dtype=torch.float64, device=A.device) if o.want_vectors else None
    q0b, ldq0 = None, max(n, 1)
    if Q0 is not None:
        if Q0.shape != (n, n) or not Q0.is_cuda:
            raise ValueError("Q0 must be an n x n CUDA tensor")
        q0b, ldq0 = _colmajor_view(Q0.to(torch.float64))
    info = Info()
    rc = lib().jacobi_eig(n, _ptr(Ab), lda, ul, _ptr(W), _ptr(Qt), max(n, 1), _ptr(q0b), ldq0,
                          _ptr(work), work.numel() * work.element_size() if work is not None else 0,
                          ctypes.byref(o), ctypes.byref(info), _stream())
    if check:
        _check(rc)
    Q = Qt.t() if Qt is not None else None
    return W, Q, info.as_dict()


def jacobi_eig_workspace(n, opts=None):
    o = opts if opts is not None else opts_default()
    return lib().jacobi_eig_workspace(n, ctypes.byref(o))


def jacobi_svd(G, opts=None, work=None, check=True):
    """Thin SVD G = U diag(S) V^T of the float64 CUDA tensor G (m x n, m >= n)
    by one-sided block Jacobi.  Returns (S, U, V, info), S descending."""
    import torch
    o = opts if opts is not None else opts_default()
    m, n = G.shape
    Gb, ldg = _colmajor_view(G)
    S = torch.empty(n, dtype=torch.float64, device=G.device)
    Ut = torch.empty((n, m), dtype=torch.float64, device=G.device) if o.want_vectors else None
    Vt = torch.empty((n, n), dtype=torch.float64, device=G.device) if o.want_vectors else None
    info = Info()
    rc = lib().jacobi_svd(m, n, _ptr(Gb), ldg, _ptr(S), _ptr(Ut), max(m, 1), _ptr(Vt), max(n, 1),
                          _ptr(work), work.numel() * work.element_size() if work is not None else 0,
                          ctypes.byref(o), ctypes.byref(info), _stream())
    if check:
        _check(rc)
    return S, (Ut.t() if Ut is not None else None), (Vt.t() if Vt is not None else None), info.as_dict()


def jacobi_svd_workspace(m, n, opts=None):
    o = opts if opts is not None else opts_default()
    return lib().jacobi_svd_workspace(m, n, ctypes.byref(o))


def jacobi_eig_batched(sizes, offsets, packed, Q0=None, opts=None, work=None, check=True, out=None,
                       info="dicts"):
    """Batched eigendecomposition.  `sizes` (host int sequence), `offsets`
    (host int64 element offsets, len = batch), `packed` a float32 or float64
    CUDA tensor holding each matrix column-major at its offset.  `out` may
    give preallocated (W, Q) float64 tensors (a call with the same sizes,
    pointers and options then replays the cached graph).  Returns (W packed by
    prefix sums of n_k, Q packed at the offsets, per-matrix info): a list of
    info dicts, or with info="array" one numpy structured array with the
    same fields (no per-matrix Python objects: large batches)."""
    import numpy as np
    import torch
    o = opts if opts is not None else opts_default()
    batch = len(sizes)
    # host arrays handed over by pointer (at least one element each)
    hn_a = np.zeros(max(batch, 1), dtype=np.int32)
    ho_a = np.zeros(max(batch, 1), dtype=np.int64)
    hn_a[:batch] = np.asarray(sizes, dtype=np.int64)[:batch]
    ho_a[:batch] = np.asarray(offsets, dtype=np.int64)[:batch]
    hn = hn_a.ctypes.data_as(_ip)
    ho = ho_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    total_w = int(hn_a[:batch].astype(np.int64).sum())
    total_q = int((ho_a[:batch] + hn_a[:batch].astype(np.int64) ** 2).max()) if batch else 0
    check_batched_args(packed, Q0, out, total_w, total_q)
    dtype = F32 if packed.dtype == torch.float32 else F64
    if out is not None:
        W, Q = out
    else:
        W = torch.empty(total_w, dtype=torch.float64, device=packed.device)
        Q = torch.empty(total_q, dtype=torch.float64, device=packed.device)
    if info not in ("dicts", "array"):
        raise ValueError("info must be 'dicts' or 'array'")
    infos = np.zeros(max(batch, 1), dtype=_info_dtype())
    rc = lib().jacobi_eig_batched(batch, hn, ho, dtype, _ptr(packed), _ptr(W), _ptr(Q), _ptr(Q0),
                                  _ptr(work), work.numel() * work.element_size() if work is not None else 0,
                                  ctypes.byref(o), infos.ctypes.data_as(ctypes.POINTER(Info)), _stream())
    if check:
        _check(rc)
    return W, Q, (infos[:batch] if info == "array" else _info_dicts(infos, batch))


def check_batched_args(packed, Q0, out, total_w, total_q):
    """Raise ValueError unless the batched call's tensors match what the
    library will read and write: `packed` float32/float64 with at least
    total_q elements, Q0 (optional) float64 with total_q, out W/Q float64
    with total_w / total_q; all contiguous CUDA tensors.  (The library takes
    raw pointers: a wrong type or a short buffer would be read or written out
    of bounds.)"""
    import torch

    todo = [(packed, "packed", (torch.float32, torch.float64), total_q)]
    if Q0 is not None:
        todo.append((Q0, "Q0", (torch.float64,), total_q))
    if out is not None:
        W, Q = out
        todo.append((W, "out W", (torch.float64,), total_w))
        if Q is not None:
            todo.append((Q, "out Q", (torch.float64,), total_q))
    for t, name, dtypes, count in todo:
        if t.dtype not in dtypes:
            raise ValueError(f"{name} must be {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < count:
            raise ValueError(f"{name} holds {t.numel()} elements, the batch needs {count}")
    for t, name, _, _ in todo:
        if not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")


def batched_workspace(sizes, dtype_f64=False, opts=None):
    """Device workspace bytes of jacobi_eig_batched for these sizes."""
    import numpy as np
    o = opts if opts is not None else opts_default()
    hn_a = np.zeros(max(len(sizes), 1), dtype=np.int32)
    hn_a[:len(sizes)] = np.asarray(sizes, dtype=np.int64)
    return int(lib().jacobi_eig_batched_workspace(len(sizes), hn_a.ctypes.data_as(_ip), F64 if dtype_f64 else F32,
                                                  ctypes.byref(o)))


def batched_tuning(dtype_f64, bucket):
    """(bs, mixed, from_file) of a size bucket (0: n<=32, 1: <=64, 2: <=128,
    3: <=192, 4: <=256) in the active tuning table."""
    bs, mixed = ctypes.c_int(), ctypes.c_int()
    rc = lib().jacobi_batched_tuning(F64 if dtype_f64 else F32, bucket, ctypes.byref(bs), ctypes.byref(mixed))
    if rc < 0 or rc > 1:
        raise JacobiError(rc, "invalid tuning query")
    return bs.value, mixed.value, rc == 1


def batched_graph_stats():
    """(cached-graph hits, graphs built) since the library was loaded."""
    h, b = ctypes.c_int(), ctypes.c_int()
    lib().jacobi_batched_graph_stats(ctypes.byref(h), ctypes.byref(b))
    return h.value, b.value


def batched_autotune(path, dtype_f64=False, per_bucket=1024, seed=0):
    """Time the candidate class parameters on a seeded calibration batch per
    size bucket, write the JSON cache to `path` and make it active.  The
    batch should fill the GPU (a few matrices per CU) so that the timings are
    throughput, as in a large call, not one matrix's latency."""
    _check(lib().jacobi_batched_autotune(F64 if dtype_f64 else F32, per_bucket, seed, str(path).encode()))


def jacobi_schedule(N, ordering=ORDER_ROUND_ROBIN):
    """The pair schedule (host computation): list of rounds of 0-based pairs."""
    pairs = (ctypes.c_int * max(N * (N - 1), 2))()
    sizes = (ctypes.c_int * max(N, 1))()
    R = lib().jacobi_schedule(N, ordering, pairs, sizes)
    if R < 0:
        raise JacobiError(R, "invalid schedule arguments")
    out, base = [], 0
    for r in range(R):
        k = sizes[r] if ordering == ORDER_ANTIDIAG else N // 2
        out.append([(pairs[2 * (base + i)], pairs[2 * (base + i) + 1]) for i in range(k)])
        base += k
    return out


def jacobi_subproblem_solve(Ahat, inner_sweeps=0):
    """Solve count independent m2 x m2 symmetric subproblems (count x m2 x m2
    float64 CUDA tensor, each read column-major = as given, symmetric).
    Returns (V, D) with V[k] orthogonal and D[k] = V[k]^T Ahat[k] V[k]
    (both as count x m2 x m2 tensors in the usual indexing)."""
    import torch
    count, m2, _ = Ahat.shape
    A = Ahat.transpose(1, 2).contiguous()  # column-major per matrix
    V = torch.empty_like(A)
    D = torch.empty_like(A)
    _check(lib().jacobi_subproblem_solve(count, m2, _ptr(A), _ptr(V), _ptr(D), inner_sweeps, _stream()))
    return V.transpose(1, 2), D.transpose(1, 2)


def jacobi_block_step(A, Q, b, pairs, V, D, fp32=False):
    """One parallel step of Alg. 2 on explicit data (in place on copies):
    returns (A_new, Q_new).  A, Q: n x n float64 CUDA tensors; V, D:
    len(pairs) x 2b x 2b tensors in the usual indexing.  fp32: the FP32
    kernels of the precision ladder compute it (jacobi_block_step32)."""
    import torch
    n = A.shape[0]
    Ac = A.t().contiguous()   # column-major A
    Qc = Q.t().contiguous() if Q is not None else None
    Vc = V.transpose(1, 2).contiguous()
    Dc = D.transpose(1, 2).contiguous()
    flat = [int(v) for pr in pairs for v in pr]
    hp = (ctypes.c_int * len(flat))(*flat)
    fn = lib().jacobi_block_step32 if fp32 else lib().jacobi_block_step
    _check(fn(n, b, _ptr(Ac), _ptr(Qc), len(pairs), hp, _ptr(Vc), _ptr(Dc), _stream()))
    torch.cuda.synchronize()
    return Ac.t(), (Qc.t() if Qc is not None else None)


def jacobi_pivot_step(A, b, pairs, V):
    """The pivoting step on explicit data (jacobi_pivot_step): A (n x n
    float64 CUDA tensor, symmetric) holds D_hat in its pair blocks, V is a
    len(pairs) x 2b x 2b float64 tensor of rotations.  Returns (A_new, V_new,
    perm) with V_new = V P, A_new's pair blocks P^T D_hat P, and perm
    (len(pairs) x 2b int32): column j of V P is column perm[j] of V."""
    import torch
    n = A.shape[0]
    Ac = A.t().contiguous()   # column-major A
    Vc = V.transpose(1, 2).contiguous()
    perm = torch.empty((len(pairs), 2 * b), dtype=torch.int32, device=A.device)
    flat = [int(v) for pr in pairs for v in pr]
    hp = (ctypes.c_int * len(flat))(*flat)
    _check(lib().jacobi_pivot_step(n, b, _ptr(Ac), len(pairs), hp, _ptr(Vc), _ptr(perm), _stream()))
    torch.cuda.synchronize()
    return Ac.t(), Vc.transpose(1, 2), perm


def jacobi_gram_blocks(G, b, pairs, fp32=False):
    """Gram blocks [G_I G_J]^T [G_I G_J] of the listed column-block pairs by the
    SVD's kernels (float64 CUDA tensor G, m x n).  Returns a len(pairs) x 2b x 2b
    tensor."""
    import torch
    m, n = G.shape
    Gb, ldg = _colmajor_view(G)
    out = torch.empty((len(pairs), 2 * b, 2 * b), dtype=torch.float64, device=G.device)
    flat = [int(v) for pr in pairs for v in pr]
    hp = (ctypes.c_int * max(len(flat), 1))(*flat)
    _check(lib().jacobi_gram_blocks(m, n, b, _ptr(Gb), ldg, len(pairs), hp, 1 if fp32 else 0, _ptr(out), _stream()))
    return out.transpose(1, 2)


def jacobi_qr(G, check=True):
    """Reduced QR G = Q R (float64 CUDA tensor G, m x n, m >= n) by the SVD's
    preprocessing kernels.  Returns (Q, R, status): R upper triangular with a
    positive diagonal; status 1 when the factorization failed."""
    import torch
    m, n = G.shape
    Gb, ldg = _colmajor_view(G)
    Qt = torch.empty((n, m), dtype=torch.float64, device=G.device)   # column-major m x n
    Rt = torch.empty((n, n), dtype=torch.float64, device=G.device)
    rc = lib().jacobi_qr(m, n, _ptr(Gb), ldg, _ptr(Qt), max(m, 1), _ptr(Rt), max(n, 1), _stream())
    if check:
        _check(rc, allow=(0, 1))
    return Qt.t(), Rt.t(), rc
