"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds no step of the Jacobi method: it only draws random
matrices of the shapes and spectra the workloads use.

* ``haar``: Haar-distributed orthogonal factor, QR of an N(0,1) matrix with the
  signs of R's diagonal moved into Q (Mezzadri 2007), sgn(0) = +1.
* ``sym_with_spectrum``: A = Q diag(lam) Q^T formed in FP64, symmetrised.
* ``eig_uniform`` / ``eig_graded``: the two eigenproblem workloads (uniform
  lam ~ U[-1, 1]; graded lam_i = +-10^(-8 i / n), i = 0..n-1, signs drawn after Q).
* ``svd_case``: G = U diag(sigma) V^T, U thin Haar m x n, V Haar n x n,
  sigma = 10^U(-6, 0).
* ``batched_case``: sizes n_k ~ U{nmin..nmax}, lam ~ N(0, 1), stored FP32.
* ``warmstart_family``: A0, B_1..B_8 symmetric with upper entries N(0, 1/n).
* ``graded_dhd``: A = D H D, H = I + E (||E||_2 = 1/2, zero diagonal), D
  diagonal and geometrically graded: positive definite with eigenvalues that
  the entries fix to high relative accuracy.
"""
import numpy as np


def haar(n, rng, m=None):
    """m x n (m >= n, default n) matrix with orthonormal columns, Haar distributed."""
    m = n if m is None else m
    X = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(X)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def sym_with_spectrum(lam, Q):
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def eig_uniform(n, seed):
    rng = np.random.default_rng(seed)
    Q = haar(n, rng)
    lam = rng.uniform(-1.0, 1.0, n)
    return sym_with_spectrum(lam, Q), lam


def eig_graded(n, seed):
    rng = np.random.default_rng(seed)
    Q = haar(n, rng)
    mag = 10.0 ** (-8.0 * np.arange(n) / n)
    sgn = rng.choice(np.array([-1.0, 1.0]), n)
    lam = mag * sgn
    return sym_with_spectrum(lam, Q), lam


def eig_normal(n, seed):
    rng = np.random.default_rng(seed)
    Q = haar(n, rng)
    lam = rng.standard_normal(n)
    return sym_with_spectrum(lam, Q), lam


def svd_case(m, n, seed):
    rng = np.random.default_rng(seed)
    U = haar(n, rng, m)
    V = haar(n, rng)
    sigma = 10.0 ** rng.uniform(-6.0, 0.0, n)
    G = np.asfortranarray((U * sigma) @ V.T)
    return G, sigma


def batched_sizes(count, seed, nmin=16, nmax=256):
    rng = np.random.default_rng(seed)
    return rng.integers(nmin, nmax + 1, size=count)


def batched_case(count, seed, nmin=16, nmax=256, dtype=np.float32):
    """Returns (sizes, offsets, packed) where matrix k is
    packed[offsets[k] : offsets[k] + n_k^2] in column-major order.  The sizes
    and the matrices come from one RNG stream in index order."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)
    packed = np.empty(int(offs[-1]), dtype=dtype)
    for k, n in enumerate(sizes):
        n = int(n)
        Q = haar(n, rng)
        lam = rng.standard_normal(n)
        A = sym_with_spectrum(lam, Q)
        packed[offs[k]:offs[k + 1]] = A.reshape(-1, order="F").astype(dtype)
    return sizes.astype(np.int32), offs, packed


def warmstart_family(seed=5, n=64, k=8):
    """A0 and B_1..B_k, each symmetric with entries on and above the diagonal
    iid N(0, 1/n), mirrored below."""
    rng = np.random.default_rng(seed)
    mats = []
    iu = np.triu_indices(n)
    for _ in range(k + 1):
        M = np.zeros((n, n))
        M[iu] = rng.standard_normal(len(iu[0])) / np.sqrt(n)
        M = M + np.triu(M, 1).T
        mats.append(np.asfortranarray(M))
    return mats[0], np.stack(mats[1:])


def warmstart_thetas(count, seed, k=8, scale=0.1):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(count, k))


def warmstart_matrices(A0, B, thetas):
    """A(theta) = A0 + sum_k theta_k B_k for each row of thetas (count x n x n)."""
    return A0[None, :, :] + np.einsum("ck,kij->cij", thetas, B)


def graded_dhd(n, seed, span):
    """A = D H D with H = I + E (E symmetric N(0, 1) scaled to ||E||_2 = 1/2,
    diagonal zero) and D = diag(10^(-span i / (n - 1))).  Returns (A, d)."""
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((n, n))
    E = 0.5 * (E + E.T)
    np.fill_diagonal(E, 0.0)
    E *= 0.5 / np.linalg.norm(E, 2)
    H = np.eye(n) + E
    d = 10.0 ** (-span * np.arange(n) / (n - 1))
    return np.asfortranarray((d[:, None] * H) * d[None, :]), d
