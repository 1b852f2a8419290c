"""FP64 reference of the learned warm start's network and training step.

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product path.

The network proposes the skew generator of a warm start for the Jacobi
eigensolver (an addition to the paper's method, which has no learned
component): theta (8) -> 256 -> 256 -> 2016 coordinates of a 64 x 64
skew-symmetric S (strictly upper entries, row-major).  Hidden layers use the
tanh form of GELU, the output layer is linear, the loss is the mean squared
error, and the optimiser is Adam (Kingma & Ba 2015).  The GPU kernels keep
BF16 copies of the weights and BF16 activations between layers; `bf16`
reproduces that rounding (round to nearest, ties to even) so the reference
can be evaluated on exactly the operands the kernels see, in FP64.
"""
import numpy as np

SIZES = (8, 256, 256, 2016)
K1PAD = 16  # the first layer's input is padded to 16 features (zeros)

C_GELU = np.sqrt(2.0 / np.pi)


def bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even); returns float64
    holding the BF16 values.  NaN stays NaN."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def bf16_bits(x):
    """The 16-bit patterns of bf16(x)."""
    return (np.asarray(bf16(x), dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def gelu(z):
    """GELU, tanh form: z/2 (1 + tanh(c (z + 0.044715 z^3))), c = sqrt(2/pi)."""
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = C_GELU * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3 * 0.044715 * z * z)


def init_params(rng, sizes=SIZES):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    Ws, bs = [], []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        Ws.append(rng.uniform(-lim, lim, size=(a, b)))
        bs.append(np.zeros(b))
    return Ws, bs


def forward(X, Ws, bs, round_acts=False):
    """Returns (Y, cache).  X: B x 8.  With round_acts the inputs of every
    layer and the saved pre-activations are rounded to BF16 (as the kernels
    store them); the activation itself is evaluated on the unrounded Z."""
    r = bf16 if round_acts else (lambda v: v)
    H = r(X)
    cache = {"H": [H], "Z": []}
    L = len(Ws)
    for l in range(L):
        Z = H @ Ws[l] + bs[l]
        if l < L - 1:
            H = r(gelu(Z))
            cache["Z"].append(r(Z))
            cache["H"].append(H)
        else:
            Y = Z
    return Y, cache


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def mse_grad(Y, T):
    return 2.0 * (Y - T) / Y.size


def backward(dY, Ws, cache, round_acts=False):
    """Gradients (dWs, dbs) of a scalar loss with dL/dY = dY.  With round_acts
    every dL/dZ (dY included) is rounded to BF16, as the kernels feed it to
    BF16 MFMA."""
    r = bf16 if round_acts else (lambda v: v)
    L = len(Ws)
    dWs, dbs = [None] * L, [None] * L
    dZ = r(dY)
    for l in range(L - 1, -1, -1):
        H = cache["H"][l]
        dWs[l] = H.T @ dZ
        dbs[l] = dZ.sum(axis=0)
        if l > 0:
            dH = dZ @ Ws[l].T
            dZ = r(dH * gelu_grad(cache["Z"][l - 1]))
    return dWs, dbs


def adam_step(p, g, m, v, lr, b1, b2, eps, step):
    """One Adam update (bias-corrected); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def skew_from_coords(c, n=64):
    """The n x n skew matrix with strictly upper entries c (row-major)."""
    S = np.zeros((n, n))
    iu = np.triu_indices(n, 1)
    S[iu] = c
    return S - S.T


def coords_from_skew(S):
    return S[np.triu_indices(S.shape[0], 1)]


def greedy_match(W):
    """Column permutation c pairing row i with column c[i]: repeatedly take the
    largest remaining |W_ij| (plain loops; ties by lowest flat index)."""
    n = W.shape[0]
    c = [-1] * n
    rows, cols = set(range(n)), set(range(n))
    A = np.abs(W)
    for _ in range(n):
        best, bi, bj = -1.0, -1, -1
        for i in sorted(rows):
            for j in sorted(cols):
                if A[i, j] > best:
                    best, bi, bj = A[i, j], i, j
        c[bi] = bj
        rows.discard(bi)
        cols.discard(bj)
    return c


def canonical_generator(Qref, Q):
    """Target of one training sample: W = Qref^T Q with its columns permuted so
    that column i is the one greedy_match pairs with Qref's column i, column
    signs with diag(W) >= 0, the column of smallest |W_jj| flipped when
    det W = -1, then S = (W - I)(W + I)^{-1} made exactly skew.
    Returns (S, W)."""
    W = Qref.T @ Q
    W = W[:, greedy_match(W)]
    s = np.where(np.diag(W) < 0.0, -1.0, 1.0)
    W = W * s
    if np.linalg.det(W) < 0.0:
        j = int(np.argmin(np.abs(np.diag(W))))
        W[:, j] = -W[:, j]
    n = W.shape[0]
    I = np.eye(n)
    S = np.linalg.solve((W + I).T, (W - I).T).T
    return 0.5 * (S - S.T), W
