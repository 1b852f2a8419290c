"""GPU parity of the one-sided block Jacobi SVD (Alg. 6) against the CPU
oracle (Hestenes one-sided Jacobi, long-double checkers).

Bars: singular values within 1e-12 sigma_max of the oracle (and of the
constructed sigma); ||G - U S V^T||_F / ||G||_F <= 1e-12 and ||V^T V - I||_F
<= 1e-12 in long double; U orthonormal on the columns with sigma > 0 to a bound
that scales like u / sigma_min (U = G Sigma^+ divides by sigma).
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_28952_amd import inputs

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def oracle_sigma(name):
    """Singular values the oracle computed for a full-size workload
    (tests/golden/make_fullsize_oracle.py), descending."""
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


@pytest.fixture(scope="module")
def jx():
    import torch
    from paper_2608_28952_amd import jacobi
    assert torch.cuda.is_available()
    jacobi.lib()
    return jacobi


def dev(a):
    import torch
    return torch.from_numpy(np.asfortranarray(a)).cuda() if a.flags.f_contiguous else torch.from_numpy(a).cuda()


def svd_gpu(jx, G, **kw):
    import torch
    check = kw.pop("check", True)
    o = jx.opts_default(**kw)
    Gt = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    S, U, V, info = jx.jacobi_svd(Gt, opts=o, check=check)
    return (S.cpu().numpy(), U.cpu().numpy() if U is not None else None,
            V.cpu().numpy() if V is not None else None, info)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("m,n,b", [(1000, 256, 64), (5000, 128, 32), (20000, 256, 64)])
def test_gram_blocks_match_oracle(jx, m, n, b, fp32):
    """The Gram-block kernels (row chunks on MFMA, fixed-order FP64 sum of the
    chunks) against the oracle's long-double G_I^T G_J, element by element.
    Bound per entry: c m u (|G_I|^T |G_J|)_ij with u the unit roundoff of the
    arithmetic (FP64, or FP32 plus the rounding of G to FP32), c = 1 (a worst
    case of the recursive sum; typical errors are ~sqrt(m) u).  m = 1000 and
    5000 leave a ragged last row chunk; columns scaled 10^U(-6, 0)."""
    import torch
    rng = np.random.default_rng(m + n + b)
    G = rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-6.0, 0.0, n)
    N = n // b
    pairs = [(0, N - 1), (1, 2)] + ([(3, N - 2)] if N >= 6 else [])
    print(f"gram m={m} n={n} b={b} fp32={fp32}", flush=True)
    out = jx.jacobi_gram_blocks(torch.from_numpy(np.asfortranarray(G)).cuda(), b, pairs, fp32=fp32).cpu().numpy()
    u = 2.0 ** -24 if fp32 else EPS
    worst = 0.0
    for k, (I, J) in enumerate(pairs):
        cols = list(range(I * b, I * b + b)) + list(range(J * b, J * b + b))
        ref = O.gram(G, cols, cols)
        absg = np.abs(G[:, cols])
        bound = (m + (2 if fp32 else 0)) * u * (absg.T @ absg)
        err = np.abs(out[k] - ref)
        assert np.all(err <= bound), (k, float(np.max(err / bound)))
        worst = max(worst, float(np.max(err / bound)))
    print(f"  largest error / bound: {worst:.2e}")


def _graded_g(m, n, seed, lo):
    """G = U diag(sigma) V^T with sigma = 10^U(lo, 0) (U, V Haar)."""
    rng = np.random.default_rng(seed)
    U, V = inputs.haar(n, rng, m), inputs.haar(n, rng)
    return (U * 10.0 ** rng.uniform(lo, 0.0, n)) @ V.T


@pytest.mark.parametrize("m,n,lo", [(300, 200, -3), (1000, 130, -6), (4000, 256, -6), (640, 384, -10)])
def test_qr_matches_oracle(jx, m, n, lo):
    """The reduced QR of the SVD's preprocessing against the oracle's long-double
    Householder QR (the factorization with diag(R) > 0 is unique): R element
    by element within 50 n u cond(G) ||G||_2 (the first-order perturbation of R
    under a backward error of c u ||G||), Q with orthonormal columns to 1e-13
    and ||G - Q R||_F <= 1e-14 ||G||_F.  cond(G) = 1e10 (lo = -10) needs the
    shifted first pass."""
    import torch
    G = _graded_g(m, n, 7 + n, lo)
    print(f"qr {m}x{n} cond 1e{-lo}", flush=True)
    Q, R, rc = jx.jacobi_qr(torch.from_numpy(np.asfortranarray(G)).cuda())
    assert rc == 0
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = O.qr(G)
    s = np.linalg.svd(G, compute_uv=False)
    bound = 50 * n * EPS * (s[0] / s[-1]) * s[0]
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)
    err = np.max(np.abs(R - Ro))
    print(f"  max |R - R_oracle| {err:.2e} (bound {bound:.2e})", flush=True)
    assert err <= bound
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
    assert np.linalg.norm(G - Q @ R) <= 1e-14 * np.linalg.norm(G)


def test_qr_rank_deficient(jx):
    """Exactly dependent columns: the Gram matrix is singular, so the first
    Cholesky either fails or leaves a tiny pivot; the shifted pass then takes
    over.  Either the call reports the failure (1) or the factors are a QR
    factorization to working accuracy; and the SVD (whose preprocessing this
    is) still matches the oracle, with one singular value at rounding level."""
    import torch
    G = np.random.default_rng(3).standard_normal((200, 64))
    G[:, 10] = G[:, 3]  # exactly dependent columns
    Q, R, rc = jx.jacobi_qr(torch.from_numpy(np.asfortranarray(G)).cuda())
    assert rc in (0, 1)
    if rc == 0:
        Q, R = Q.cpu().numpy(), R.cpu().numpy()
        print(f"rank deficient: ||G - QR|| / ||G|| {np.linalg.norm(G - Q @ R) / np.linalg.norm(G):.2e}, "
              f"||Q^T Q - I|| {np.linalg.norm(Q.T @ Q - np.eye(64)):.2e}")
        assert np.linalg.norm(G - Q @ R) <= 1e-14 * np.linalg.norm(G)
    S, U, V, info = svd_gpu(jx, G)
    assert info["status"] == 0
    ora = O.svd(G)
    assert np.max(np.abs(S - ora.S)) <= 1e-12 * ora.S[0] and S[-1] <= 1e-14 * S[0]
    res, ov, _ = O.check_svd(G, S, U, V)
    assert res <= 1e-12 and ov <= 1e-12


@pytest.mark.parametrize("precondition", [-1, 0])
@pytest.mark.parametrize("m,n", [(100, 40), (256, 128), (300, 200), (1000, 64), (130, 130)])
def test_svd_parity_with_oracle(jx, m, n, precondition):
    rng = np.random.default_rng(m + n)
    G = rng.standard_normal((m, n))
    print(f"svd {m}x{n} precondition={precondition}", flush=True)
    S, U, V, info = svd_gpu(jx, G, precondition=precondition)
    assert info["status"] == 0
    ora = O.svd(G)
    assert np.max(np.abs(S - ora.S)) <= 1e-12 * ora.S[0]
    res, ov, ou = O.check_svd(G, S, U, V)
    assert res <= 1e-12 and ov <= 1e-12 and ou <= 1e-12, (res, ov, ou)


@pytest.mark.parametrize("m,n", [(512, 128), (2048, 256)])
def test_svd_constructed_log_uniform_sigma(jx, m, n):
    """G = U diag(sigma) V^T, sigma = 10^U(-6, 0): the C3 recipe at reduced size."""
    G, sigma = inputs.svd_case(m, n, 3)
    S, U, V, info = svd_gpu(jx, G)
    assert info["status"] == 0
    ref = np.sort(sigma)[::-1]
    assert np.max(np.abs(S - ref)) <= 1e-12 * ref[0]
    ora = O.svd(G)
    assert np.max(np.abs(S - ora.S)) <= 1e-12 * ref[0]
    rel = np.max(np.abs(S - ora.S) / ora.S)
    print(f"max relative sigma error vs oracle: {rel:.2e}")
    assert rel <= 1e-8  # reported statistic; tiny sigma ~1e-6 lose ~u/sigma relative
    res, ov, ou = O.check_svd(G, S, U, V)
    assert res <= 1e-12 and ov <= 1e-12
    assert ou <= 1e-12 / ref[-1]


@pytest.mark.parametrize("precondition", [0, -1])
def test_svd_sweep_cap_with_refinement(jx, precondition):
    """opts.max_sweeps bounds the sweeps up to the refinement of V, which
    runs inside the quadratic phase (the sweeps after a refinement may run
    past the cap, as after a refinement at convergence): with a cap below
    the sweep that starts it, the solve stops at the cap with status 1.  The
    full solve refines after its third-last sweep (one rotating and one
    checking sweep follow)."""
    G, sigma = inputs.svd_case(2048, 256, 3)
    S, _, _, info = svd_gpu(jx, G, precondition=precondition)
    assert info["status"] == 0, info
    ref = np.sort(sigma)[::-1]
    assert np.max(np.abs(S - ref)) <= 1e-12 * ref[0]
    n_sw = info["sweeps"]
    print(f"svd 2048 x 256 precondition={precondition}: {n_sw} sweeps", flush=True)
    for cap in (n_sw - 3, n_sw // 2):
        _, _, _, ic = svd_gpu(jx, G, precondition=precondition, max_sweeps=cap, check=False)
        assert ic["status"] == 1 and ic["sweeps"] == cap, (cap, ic)


def test_svd_edge_cases(jx):
    rng = np.random.default_rng(5)
    # a zero column: sigma = 0 and a zero U column
    G = rng.standard_normal((90, 30))
    G[:, 7] = 0.0
    S, U, V, info = svd_gpu(jx, G)
    assert info["status"] == 0 and S[-1] == 0.0 and np.all(U[:, -1] == 0.0)
    # orthonormal columns: all sigma = 1
    Q = inputs.haar(50, rng, 200)
    S, U, V, info = svd_gpu(jx, Q)
    assert np.max(np.abs(S - 1.0)) <= 1e-14
    # n = 1
    g = rng.standard_normal((20, 1))
    S, U, V, info = svd_gpu(jx, g)
    assert abs(S[0] - np.linalg.norm(g)) <= 1e-14 * np.linalg.norm(g)
    # values only
    G = rng.standard_normal((64, 48))
    Sv, Uv, Vv, info = svd_gpu(jx, G, want_vectors=0)
    assert Uv is None and np.max(np.abs(Sv - O.svd(G).S)) <= 1e-12 * Sv[0]
    # not converged / m < n
    G = rng.standard_normal((300, 200))
    _, _, _, info = svd_gpu(jx, G, max_sweeps=1, refine=0, check=False)
    assert info["status"] == 1
    import torch
    with pytest.raises(Exception):
        jx.jacobi_svd(torch.zeros((3, 5), dtype=torch.float64, device="cuda"))
    # the zero matrix (the QR preprocessing cannot factor it: the plain solve
    # runs), with and without vectors
    for wv in (1, 0):
        S, U, V, info = svd_gpu(jx, np.zeros((300, 130)), want_vectors=wv)
        assert info["status"] == 0 and np.all(S == 0.0)
        if wv:
            assert np.all(U == 0.0) and np.linalg.norm(V.T @ V - np.eye(130)) <= 1e-13
    # n = 0, and a non-finite entry
    S, U, V, info = jx.jacobi_svd(torch.zeros((7, 0), dtype=torch.float64, device="cuda"))
    assert S.numel() == 0 and info["status"] == 0
    G = rng.standard_normal((200, 64))
    G[3, 5] = np.nan
    _, _, _, info = svd_gpu(jx, G, check=False)
    assert info["status"] == 2


def test_svd_deterministic(jx):
    G = np.random.default_rng(8).standard_normal((400, 160))
    a = svd_gpu(jx, G)
    b = svd_gpu(jx, G)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("precondition", [-1, 0])
def test_svd_full_size_16384x2048(jx, precondition):
    """The full workload (m = 16384, n = 2048, sigma log-uniform in [1e-6, 1],
    seed 3), with QR preprocessing (default) and without: the oracle's sigma of
    the same matrix (fixture) and the full long-double checks."""
    m, n = 16384, 2048
    G, sigma = inputs.svd_case(m, n, 3)
    print(f"svd 16384x2048 precondition={precondition}", flush=True)
    S, U, V, info = svd_gpu(jx, G, precondition=precondition)
    assert info["status"] == 0, info
    ref = np.sort(sigma)[::-1]
    ora = oracle_sigma("svd_16384x2048_seed3.txt")
    assert np.max(np.abs(S - ora)) <= 1e-12 * ora[0]
    assert np.max(np.abs(S - ref)) <= 1e-12 * ref[0]
    rel_o, rel = np.max(np.abs(S - ora) / ora), np.max(np.abs(S - ref) / ref)
    res, ov, ou = O.check_svd(G, S, U, V)
    print(f"svd full: sweeps {info['sweeps']} max rel sigma err vs oracle {rel_o:.2e}, vs construction {rel:.2e}; "
          f"residual {res:.2e} V orth {ov:.2e} U orth {ou:.2e}", flush=True)
    assert rel_o <= 1e-8  # reported statistic (A20); tiny sigma ~1e-6 lose ~u/sigma relative
    assert res <= 1e-12 and ov <= 1e-12 and ou <= 1e-12 / ref[-1], (res, ov, ou)


@pytest.mark.parametrize("m,n", [(512, 128), (1000, 64), (2048, 256)])
def test_svd_mixed_fp32_matches_oracle(jx, m, n):
    G, sigma = inputs.svd_case(m, n, 30 + n)
    S, U, V, info = svd_gpu(jx, G, precision=jx.PREC_MIXED_FP32)
    assert info["status"] == 0, info
    assert info["sweeps_by_prec"][1] > 0
    ora = O.svd(G)
    assert np.max(np.abs(S - ora.S)) <= 1e-12 * ora.S[0]
    print(f"svd mixed {m}x{n}: sweeps {info['sweeps_by_prec']}, max rel {np.max(np.abs(S - ora.S) / ora.S):.2e}")
    res, ov, ou = O.check_svd(G, S, U, V)
    assert res <= 1e-12 and ov <= 1e-12 and ou <= 1e-12 / ora.S[-1]


def test_svd_full_size_mixed_fp32(jx):
    m, n = 16384, 2048
    G, sigma = inputs.svd_case(m, n, 3)
    S, U, V, info = svd_gpu(jx, G, precision=jx.PREC_MIXED_FP32)
    assert info["status"] == 0, info
    ref = np.sort(sigma)[::-1]
    rel = np.max(np.abs(S - ref) / ref)
    print(f"svd full mixed: sweeps {info['sweeps_by_prec']} max rel sigma err {rel:.2e}")
    assert np.max(np.abs(S - ref)) <= 1e-12 * ref[0]
    # the FP32 phase ends near 2 u32 cond(G) (cond 1e6 here): no more sweeps
    # in all than plain FP64 takes (38); running it on to 1e-5 took 46
    assert sum(info["sweeps_by_prec"]) <= 40, info
    ora = oracle_sigma("svd_16384x2048_seed3.txt")
    assert np.max(np.abs(S - ora)) <= 1e-12 * ora[0]
    res, ov, ou = O.check_svd(G, S, U, V)
    print(f"  residual {res:.2e} V orth {ov:.2e} U orth {ou:.2e}", flush=True)
    assert res <= 1e-12 and ov <= 1e-12 and ou <= 1e-12 / ref[-1], (res, ov, ou)
