"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these tests touches the GPU library.  Each test pins the oracle to
something other than itself: values printed in the paper (tests/golden/),
closed forms, invariants, high-precision arithmetic (mpmath, 50 digits),
special cases with known answers, and LAPACK through numpy.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_28952_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# --------------------------------------------------------------------------
# Orderings: Alg. 3 against the printed list L (eq. parallel_list, §3)
# --------------------------------------------------------------------------

def printed_L():
    groups = []
    for row in _read_rows("parallel_list_P8.txt"):
        groups.append({tuple(int(x) - 1 for x in tok.split("-")) for tok in row})
    return groups


def test_alg3_matches_printed_list():
    L = [set(g) for g in O.antidiag_list(8)]
    P = printed_L()
    # The paper prints Alg. 3's groups in the order K = 1, 0, 7, 6, ..., 2:
    # printed group g (1-based) is Alg. 3's group K = (2 - g) mod 8.
    for g in range(1, 9):
        assert P[g - 1] == L[(2 - g) % 8], g
    assert sorted(map(sorted, P)) == sorted(map(sorted, L))


def test_alg3_group_sizes_alternate():
    sizes = [len(g) for g in O.antidiag_list(8)]
    assert sorted(sizes) == [3, 3, 3, 3, 4, 4, 4, 4]
    assert all(sizes[k] != sizes[(k + 1) % 8] for k in range(8))


def test_printed_labels_match_list():
    rows = _read_rows("disjoint_labels_P8.txt")
    P = printed_L()
    for I, row in enumerate(rows):
        for off, lab in enumerate(row):
            J = I + 1 + off
            assert (I, J) in P[int(lab) - 1]


def _transformation_labels(group, P=8):
    """Label of block (I, J): the transformation acting on block row I (left)
    and the one acting on block column J (right)."""
    who = {}
    for t, (a, b) in enumerate(group, start=1):
        who[a] = t
        who[b] = t
    out = []
    for I in range(P):
        row = []
        for J in range(I, P):
            l, r = who.get(I), who.get(J)
            if l is not None and l == r:
                row.append(str(l))
            else:
                row.append(("_" if l is None else str(l)) + ("_" if r is None else str(r)))
        out.append(row)
    return out


@pytest.mark.parametrize("fname,g", [("group_one_transformations_P8.txt", 1),
                                     ("group_two_transformations_P8.txt", 2)])
def test_update_pattern_matches_paper(fname, g):
    rows = _read_rows(fname)
    # label order = printed order within the group
    printed = [[tuple(int(x) - 1 for x in tok.split("-")) for tok in row]
               for row in _read_rows("parallel_list_P8.txt")]
    assert _transformation_labels(printed[g - 1]) == rows


@pytest.mark.parametrize("N", [2, 4, 6, 8, 16, 64, 5, 7])
def test_round_robin_covers_each_pair_once(N):
    R = O.rr_list(N)
    seen = set()
    for rnd in R:
        used = set()
        for (I, J) in rnd:
            assert 0 <= I < J < N
            assert I not in used and J not in used
            used |= {I, J}
            assert (I, J) not in seen
            seen.add((I, J))
        if N % 2 == 0:
            assert len(rnd) == N // 2
    assert len(seen) == N * (N - 1) // 2
    assert len(R) == (N - 1 if N % 2 == 0 else N)


@pytest.mark.parametrize("N", list(range(2, 41)))
def test_schedules_equal_the_scan_of_their_definition(N):
    """The group of Alg. 3 (pairs with I + J = K mod P, in increasing I) and the
    even-N round-robin built on it, against a plain scan over all pairs."""
    def scan(P):
        return [[(I - 1, J - 1) for I in range(1, P) for J in range(I + 1, P + 1) if (I + J) % P == K % P]
                for K in range(P)]
    assert O.antidiag_list(N) == scan(N)
    if N % 2 == 0:
        M = N - 1
        want = [g + [(I - 1, N - 1) for I in range(1, M + 1) if (2 * I) % M == K % M] if M > 0 else []
                for K, g in enumerate(scan(M) if M > 1 else [[]])]
        assert O.rr_list(N) == want


def test_round_robin_n64_shape():
    R = O.rr_list(64)
    assert len(R) == 63 and all(len(r) == 32 for r in R)


# --------------------------------------------------------------------------
# Scalar Jacobi eigensolver (Alg. 1 with b = 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("a,b,d", [(2.0, 1.0, -1.0), (1.0, 0.5, 1.0), (0.0, 3.0, 0.0),
                                   (1e-3, 1e-9, 2e-3), (-5.0, 2.0, 7.0)])
@pytest.mark.parametrize("order", [0, 1])
def test_eig_2x2_closed_form(a, b, d, order):
    A = np.array([[a, b], [b, d]])
    r = O.eig(A, order=order)
    m, h = 0.5 * (a + d), math.hypot(0.5 * (a - d), b)
    assert r.status == 0
    np.testing.assert_allclose(r.W, [m - h, m + h], rtol=0, atol=4 * EPS * max(abs(a), abs(b), abs(d)))
    # one rotation diagonalises a 2x2 exactly; eigenvector check
    for k in range(2):
        v = r.Q[:, k]
        np.testing.assert_allclose(A @ v, r.W[k] * v, atol=8 * EPS * (abs(a) + abs(b) + abs(d)))
    assert r.rotations <= 1


def _smith_3x3(A):
    """O. K. Smith, 'Eigenvalues of a symmetric 3x3 matrix', CACM 4(4), 1961."""
    q = np.trace(A) / 3.0
    p1 = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2 * p1
    p = math.sqrt(p2 / 6.0)
    B = (A - q * np.eye(3)) / p
    r = np.linalg.det(B) / 2.0
    r = min(1.0, max(-1.0, r))
    phi = math.acos(r) / 3.0
    l1 = q + 2 * p * math.cos(phi)
    l3 = q + 2 * p * math.cos(phi + 2 * math.pi / 3)
    l2 = 3 * q - l1 - l3
    return np.sort([l1, l2, l3])


@pytest.mark.parametrize("seed", range(6))
def test_eig_3x3_closed_form(seed):
    rng = np.random.default_rng(100 + seed)
    Q = inputs.haar(3, rng)
    lam = np.array([-1.0, 0.3, 2.0]) * (1 + seed)
    A = inputs.sym_with_spectrum(lam, Q)
    r = O.eig(A)
    np.testing.assert_allclose(r.W, _smith_3x3(A), rtol=0, atol=1e-13 * (1 + seed))
    np.testing.assert_allclose(r.W, lam, rtol=0, atol=1e-14 * (1 + seed) * 4)


def test_eig_mpmath_50_digits():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7)
    for n in (4, 7, 12):
        X = rng.standard_normal((n, n))
        A = X + X.T
        ev = mpmath.eigsy(mpmath.matrix(A.tolist()), eigvals_only=True)
        ref = np.sort(np.array([float(x) for x in ev]))
        r = O.eig(A, order=1)
        nrm = np.linalg.norm(A, 2)
        assert np.max(np.abs(r.W - ref)) <= 8 * n * EPS * nrm


@pytest.mark.parametrize("n,kind", [(64, "uniform"), (64, "graded"), (128, "uniform")])
def test_eig_known_spectrum_and_invariants(n, kind):
    A, lam = (inputs.eig_uniform(n, 11) if kind == "uniform" else inputs.eig_graded(n, 12))
    r = O.eig(A, order=1)
    assert r.status == 0
    nrm = np.max(np.abs(lam))
    # Weyl: each eigenvalue moves by at most the backward error ~ n u ||A||_2
    assert np.max(np.abs(r.W - np.sort(lam))) <= n * EPS * nrm
    res, orth, dtr, dfro = O.check_eig(A, r.W, r.Q)
    # the A = Q D Q^T invariants at the 1e-12 bar, measured in long double
    assert res <= 1e-13 and orth <= 1e-12
    assert abs(dtr) <= n * EPS * np.sum(np.abs(lam))
    assert abs(dfro) <= n * EPS
    # numpy / LAPACK as a second, independent reference
    assert np.max(np.abs(r.W - np.linalg.eigvalsh(A))) <= 1e-12 * nrm


def test_eig_orders_agree():
    A, _ = inputs.eig_uniform(40, 3)
    r0 = O.eig(A, order=0)
    r1 = O.eig(A, order=1)
    r2 = O.eig(A, order=1, nthreads=4)
    nrm = np.max(np.abs(r0.W))
    assert np.max(np.abs(r0.W - r1.W)) <= 1e-13 * nrm
    assert np.max(np.abs(r1.W - r2.W)) <= 1e-13 * nrm
    for r in (r0, r1, r2):
        res, orth, _, _ = O.check_eig(A, r.W, r.Q)
        assert res <= 1e-13 and orth <= 1e-13


def test_per_rotation_identity():
    """§1: each 2x2 rotation lowers off^2 by exactly 2 a_pq^2 (to rounding)."""
    A, _ = inputs.eig_uniform(24, 5)
    for order in (0, 1):
        r = O.eig(A, order=order, check_rotations=True)
        assert r.rotations > 0
        assert r.rot_identity <= 1e-12


def test_diagonal_input_is_fixed_point():
    d = np.array([3.0, -1.0, 2.0, 0.5, -7.0])
    A = np.diag(d)
    r = O.eig(A)
    assert r.rotations == 0 and r.sweeps == 0
    np.testing.assert_array_equal(r.W, np.sort(d))
    perm = np.argsort(d, kind="stable")
    np.testing.assert_array_equal(r.Q, np.eye(5)[:, perm])


def test_identity_plus_rank_one():
    rng = np.random.default_rng(9)
    u = rng.standard_normal(30)
    A = np.eye(30) + np.outer(u, u)
    r = O.eig(A)
    expect = np.ones(30)
    expect[-1] = 1 + u @ u
    np.testing.assert_allclose(r.W, expect, rtol=0, atol=30 * EPS * (1 + u @ u))


def test_block_diagonal_decouples():
    A1, l1 = inputs.eig_uniform(7, 1)
    A2, l2 = inputs.eig_uniform(5, 2)
    A = np.zeros((12, 12))
    A[:7, :7] = A1
    A[7:, 7:] = A2
    r = O.eig(A)
    np.testing.assert_allclose(r.W, np.sort(np.concatenate([O.eig(A1).W, O.eig(A2).W])), atol=1e-14)
    # no rotation ever mixes the blocks (their coupling entries are exact zeros)
    for k in range(12):
        v = r.Q[:, k]
        assert np.all(v[:7] == 0) or np.all(v[7:] == 0)


def test_metamorphic_shift_negate_permute():
    A, _ = inputs.eig_uniform(32, 4)
    w = O.eig(A).W
    nrm = np.max(np.abs(w))
    np.testing.assert_allclose(O.eig(A + 2.5 * np.eye(32)).W, w + 2.5, atol=1e-13 * (nrm + 2.5))
    np.testing.assert_allclose(O.eig(-A).W, -w[::-1], atol=1e-13 * nrm)
    p = np.random.default_rng(1).permutation(32)
    np.testing.assert_allclose(O.eig(A[np.ix_(p, p)]).W, w, atol=1e-13 * nrm)


def test_resume_from_intermediate_q():
    A, _ = inputs.eig_uniform(48, 8)
    full = O.eig(A)
    part = O.eig(A, max_sweeps=2)
    assert part.status == 1
    # part.Q holds the (sorted) iterate after 2 sweeps; restart from it
    res = O.eig(A, Q0=part.Q)
    assert res.status == 0
    assert np.max(np.abs(res.W - full.W)) <= 1e-13
    assert res.sweeps < full.sweeps


def test_status_codes():
    A, _ = inputs.eig_uniform(16, 1)
    assert O.eig(A, max_sweeps=1).status == 1
    B = A.copy()
    B[3, 4] = np.nan
    assert O.eig(B).status == 2
    assert O.eig(np.zeros((0, 0))).status == 0


# --------------------------------------------------------------------------
# One-sided Jacobi SVD (Alg. 6 with b = 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(20, 12), (64, 64), (100, 30)])
def test_svd_constructed_sigma(m, n):
    G, sigma = inputs.svd_case(m, n, 21)
    r = O.svd(G)
    assert r.status == 0
    s_ref = np.sort(sigma)[::-1]
    assert np.max(np.abs(r.S - s_ref)) <= 10 * n * EPS
    np.testing.assert_allclose(r.S, np.linalg.svd(G, compute_uv=False), rtol=0, atol=10 * n * EPS)
    res, ov, ou = O.check_svd(G, r.S, r.U, r.V)
    assert res <= 1e-13 and ov <= 1e-12
    # U's orthogonality degrades like u / sigma_min for the tiny sigmas
    assert ou <= 1e-13 / s_ref[-1] * 10


def test_svd_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(3)
    G = rng.standard_normal((9, 6))
    ref = np.array([float(x) for x in mpmath.svd_r(mpmath.matrix(G.tolist()), compute_uv=False)])
    r = O.svd(G)
    np.testing.assert_allclose(r.S, np.sort(ref)[::-1], rtol=0, atol=50 * EPS * ref.max())


def test_svd_orthonormal_columns_and_rank_deficient():
    rng = np.random.default_rng(4)
    G = inputs.haar(8, rng, 20)
    r = O.svd(G)
    np.testing.assert_allclose(r.S, np.ones(8), atol=1e-14)
    H = rng.standard_normal((15, 6))
    H[:, 2] = 0.0
    r = O.svd(H)
    assert r.S[-1] == 0.0
    assert np.all(r.U[:, -1] == 0.0)


def test_svd_squares_are_gram_eigenvalues():
    G, _ = inputs.svd_case(40, 10, 5)
    G = G + np.asfortranarray(np.eye(40, 10))  # well conditioned
    s = O.svd(G).S
    w = O.eig(G.T @ G).W
    np.testing.assert_allclose(np.sort(s ** 2), w, rtol=1e-12)


# --------------------------------------------------------------------------
# Block step (Alg. 2 formulas) against the composite product V^T A V
# --------------------------------------------------------------------------

def _composite(n, b, pairs, Vhat):
    V = np.eye(n)
    for (I, J), Vh in zip(pairs, Vhat):
        idx = np.r_[I * b:(I + 1) * b, J * b:(J + 1) * b]
        V[np.ix_(idx, idx)] = Vh
    return V


@pytest.mark.parametrize("N,b,rnd", [(4, 3, 0), (6, 2, 2), (5, 2, 1)])
def test_block_step_equals_composite_rotation(N, b, rnd):
    n = N * b
    rng = np.random.default_rng(N * 10 + b)
    A, _ = inputs.eig_uniform(n, 30 + N)
    Q = inputs.haar(n, rng)
    pairs = O.rr_list(N)[rnd]
    Vhat = [inputs.haar(2 * b, rng) for _ in pairs]
    Dhat = [np.diag(rng.standard_normal(2 * b)) for _ in pairs]
    An, Qn = O.block_step(A, Q, b, pairs, Vhat, Dhat)
    V = _composite(n, b, pairs, Vhat)
    ref = V.T @ A @ V
    for (I, J), D in zip(pairs, Dhat):
        idx = np.r_[I * b:(I + 1) * b, J * b:(J + 1) * b]
        ref[np.ix_(idx, idx)] = D
    np.testing.assert_allclose(An, ref, rtol=0, atol=1e-14 * n)
    np.testing.assert_allclose(Qn, Q @ V, rtol=0, atol=1e-14 * n)


def test_block_step_identity_rotations_keep_a():
    n, b = 12, 3
    A, _ = inputs.eig_uniform(n, 2)
    pairs = O.rr_list(4)[1]
    An, Qn = O.block_step(A, np.eye(n), b, pairs, [np.eye(2 * b)] * len(pairs))
    np.testing.assert_array_equal(An, A)
    np.testing.assert_array_equal(Qn, np.eye(n))


# --------------------------------------------------------------------------
# Cayley map
# --------------------------------------------------------------------------

def test_cayley_identities():
    rng = np.random.default_rng(0)
    n = 10
    X = rng.standard_normal((n, n)) * 0.3
    S = X - X.T
    W = O.cayley(S)
    np.testing.assert_allclose(W.T @ W, np.eye(n), atol=1e-14 * n)
    np.testing.assert_allclose(O.cayley(-S), W.T, atol=1e-14 * n)
    np.testing.assert_array_equal(O.cayley(np.zeros((n, n))), np.eye(n))
    np.testing.assert_allclose(O.cayley_inverse(W), S, atol=1e-13 * n)
    s = 0.7
    W2 = O.cayley(np.array([[0.0, s], [-s, 0.0]]))
    ref = np.array([[1 - s * s, 2 * s], [-2 * s, 1 - s * s]]) / (1 + s * s)
    np.testing.assert_allclose(W2, ref, atol=4 * EPS)


# --------------------------------------------------------------------------
# Checkers
# --------------------------------------------------------------------------

def test_checker_detects_errors():
    A, lam = inputs.eig_uniform(20, 6)
    r = O.eig(A)
    good = O.check_eig(A, r.W, r.Q)
    assert good[0] < 1e-14 and good[1] < 1e-13
    Qb = r.Q.copy()
    Qb[:, 3] *= -1.0
    Qb[:, [4, 5]] = Qb[:, [5, 4]]  # swapped vectors: residual must see it
    bad = O.check_eig(A, r.W, Qb)
    assert bad[0] > 1e-3 and bad[1] < 1e-13
    samp = O.check_eig_sampled(A, r.W, r.Q, [0, 3, 19])
    assert samp[0] < 1e-14 and samp[1] < 1e-13
    assert O.check_offnorm(np.diag([1.0, 2.0])) == 0.0
    assert abs(O.check_offnorm(np.array([[0.0, 3.0], [4.0, 0.0]])) - 5.0) < 1e-15


# --------------------------------------------------------------------------
# Checkers: planted errors of known size must be reported at that size
# --------------------------------------------------------------------------
# Each case perturbs an exact decomposition by a rank-one or 2 x 2 change whose
# effect on the measured quantity has a closed form, and requires the checker
# to report that value (relative 1e-3, far above the ~1e-14 rounding of the
# unperturbed decomposition).  A checker that dropped a term, a column or a
# sample, or returned zeros, fails here.

def _eig_exact(n, seed):
    A, _ = inputs.eig_uniform(n, seed)
    r = O.eig(A)
    assert r.status == 0
    return A, r.W, r.Q


def _rot(Q, c, d, phi):
    """Columns c, d of Q rotated by phi: q_c' = cos q_c + sin q_d, q_d' = -sin q_c + cos q_d."""
    Q = Q.copy()
    qc, qd = Q[:, c].copy(), Q[:, d].copy()
    Q[:, c] = math.cos(phi) * qc + math.sin(phi) * qd
    Q[:, d] = -math.sin(phi) * qc + math.cos(phi) * qd
    return Q


def _close(got, want, rel=1e-3):
    assert abs(got - want) <= rel * abs(want), (got, want)


def test_check_eig_reports_planted_errors():
    A, W, Q = _eig_exact(24, 11)
    fro = np.linalg.norm(A)
    # column c scaled by (1 + e): Q^T Q - I gains (2e + e^2) at (c, c); the
    # residual gains lambda_c (2e + e^2) q_c q_c^T
    e, c = 1e-6, 5
    Qs = Q.copy()
    Qs[:, c] *= 1.0 + e
    res, orth, _, _ = O.check_eig(A, W, Qs)
    _close(orth, 2 * e + e * e)
    _close(res, abs(W[c]) * (2 * e + e * e) / fro)
    # two columns rotated by phi: still orthogonal, residual sqrt(2) |l_c - l_d| |sin phi|
    c, d, phi = 3, 17, 1e-5
    res, orth, _, _ = O.check_eig(A, W, _rot(Q, c, d, phi))
    assert orth < 1e-13
    _close(res, math.sqrt(2) * abs(W[c] - W[d]) * abs(math.sin(phi)) / fro)
    # an eigenvalue moved by delta: residual |delta| / ||A||_F, trace off by -delta
    Wd = W.copy()
    Wd[7] += 3e-7
    res, orth, dtr, _ = O.check_eig(A, Wd, Q)
    _close(res, 3e-7 / fro)
    _close(dtr, -3e-7, rel=1e-6)


def test_check_eig_sampled_reports_planted_errors():
    A, W, Q = _eig_exact(24, 12)
    fro = np.linalg.norm(A)
    c, d, phi = 4, 9, 2e-6
    Qr = _rot(Q, c, d, phi)
    # A q_c' - l_c q_c' = sin(phi) (l_d - l_c) q_d
    res, orth = O.check_eig_sampled(A, W, Qr, [0, c, 20])
    _close(res, abs(math.sin(phi) * (W[d] - W[c])) / fro)
    assert orth < 1e-13
    # a column outside the sample is not seen; inside it is
    res, _ = O.check_eig_sampled(A, W, Qr, [0, 1, 20])
    assert res < 1e-14
    e = 4e-7
    Qs = Q.copy()
    Qs[:, 11] *= 1.0 + e
    res, orth = O.check_eig_sampled(A, W, Qs, [2, 11])
    _close(orth, 2 * e + e * e)
    assert res < 1e-14  # a scaled eigenvector still satisfies A q = l q
    Wd = W.copy()
    Wd[2] -= 5e-8
    res, orth = O.check_eig_sampled(A, Wd, Q, [2, 11])
    _close(res, 5e-8 / fro)


def _svd_exact(m, n, seed):
    G, _ = inputs.svd_case(m, n, seed)
    r = O.svd(G)
    assert r.status == 0
    return G, r.S, r.U, r.V


def test_check_svd_reports_planted_errors():
    G, S, U, V = _svd_exact(40, 16, 13)
    fro = np.linalg.norm(G)
    res, ov, ou = O.check_svd(G, S, U, V)
    assert res < 1e-14 and ov < 1e-13 and ou < 1e-13
    # sigma_c moved by delta: G - U S' V^T = -delta u_c v_c^T
    Sd = S.copy()
    Sd[3] += 2e-7
    res, ov, ou = O.check_svd(G, Sd, U, V)
    _close(res, 2e-7 / fro)
    assert ov < 1e-13 and ou < 1e-13
    # V column scaled: ||V^T V - I|| = 2e + e^2, residual sigma_c e
    e = 1e-6
    Vs = V.copy()
    Vs[:, 5] *= 1.0 + e
    res, ov, ou = O.check_svd(G, S, U, Vs)
    _close(ov, 2 * e + e * e)
    _close(res, S[5] * e / fro)
    # U column scaled: ||U^T U - I|| = 2e + e^2
    Us = U.copy()
    Us[:, 6] *= 1.0 + e
    res, ov, ou = O.check_svd(G, S, Us, V)
    _close(ou, 2 * e + e * e)
    _close(res, S[6] * e / fro)
    # two U columns rotated by phi: U stays orthonormal, residual
    # ||(I - R) diag(s_c, s_d)||_F = sqrt((s_c^2 + s_d^2)(2 - 2 cos phi))
    c, d, phi = 1, 12, 1e-4
    res, ov, ou = O.check_svd(G, S, _rot(U, c, d, phi), V)
    assert ou < 1e-13
    _close(res, math.sqrt((S[c] ** 2 + S[d] ** 2) * (2 - 2 * math.cos(phi))) / fro)


def test_check_svd_zero_sigma_columns_left_out():
    G, S, U, V = _svd_exact(30, 8, 14)
    S0, U0 = S.copy(), U.copy()
    S0[-1] = 0.0
    U0[:, -1] = 0.0
    _, _, ou = O.check_svd(G, S0, U0, V)
    assert ou < 1e-13


def test_check_svd_sampled_reports_planted_errors():
    G, S, U, V = _svd_exact(40, 16, 15)
    fro = np.linalg.norm(G)
    cols = [0, 5, 11]
    res, wv, wu = O.check_svd_sampled(G, S, U, V, cols)
    assert res < 1e-14 and wv < 1e-13 and wu < 1e-13
    Sd = S.copy()
    Sd[5] -= 4e-7
    res, _, _ = O.check_svd_sampled(G, Sd, U, V, cols)
    _close(res, 4e-7 / fro)
    e = 2e-6
    Vs = V.copy()
    Vs[:, 11] *= 1.0 + e
    res, wv, _ = O.check_svd_sampled(G, S, U, Vs, cols)
    _close(wv, 2 * e + e * e)
    _close(res, S[11] * e / fro)
    Us = U.copy()
    Us[:, 0] *= 1.0 + e
    res, _, wu = O.check_svd_sampled(G, S, Us, V, cols)
    _close(wu, 2 * e + e * e)
    _close(res, S[0] * e / fro)
    # outside the sample: not seen
    res, wv, wu = O.check_svd_sampled(G, Sd, U, V, [0, 11])
    assert res < 1e-14


def test_full_checker_agrees_with_sampled_on_all_columns():
    # the two checkers share no code: on every column the sampled maxima are
    # bounded by the full Frobenius norms, and a single planted error shows in both
    A, W, Q = _eig_exact(20, 16)
    Qs = Q.copy()
    Qs[:, 8] *= 1.0 + 3e-6
    full = O.check_eig(A, W, Qs)
    samp = O.check_eig_sampled(A, W, Qs, list(range(20)))
    _close(samp[1], full[1])
    assert samp[0] <= full[0] * 1.0001


# --------------------------------------------------------------------------
# Gram blocks (eq. SVD_subproblem, §6)
# --------------------------------------------------------------------------

def test_gram_exact_on_integers():
    # small integer entries: every product and partial sum is exact in
    # binary floating point, so the Gram block equals the integer product
    rng = np.random.default_rng(21)
    m, n = 300, 20
    Gi = rng.integers(-50, 51, size=(m, n))
    ca, cb = [0, 3, 7, 19, 2], [5, 5, 1, 18]
    ref = Gi[:, ca].T.astype(np.int64) @ Gi[:, cb].astype(np.int64)
    out = O.gram(Gi.astype(np.float64), ca, cb)
    np.testing.assert_array_equal(out, ref.astype(np.float64))


def test_gram_matches_numpy_within_bound_and_is_symmetric():
    rng = np.random.default_rng(22)
    m, n = 1000, 24
    G = rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-6, 0, n)
    I, J = list(range(0, 12)), list(range(12, 24))
    cols = I + J
    out = O.gram(G, cols, cols)
    ref = G[:, cols].T @ G[:, cols]
    bound = m * EPS * (np.abs(G[:, cols]).T @ np.abs(G[:, cols]))
    assert np.all(np.abs(out - ref) <= bound)
    np.testing.assert_array_equal(out, out.T)
    np.testing.assert_array_equal(O.gram(G, I, J), O.gram(G, J, I).T)
    # orthonormal columns: the identity
    Qh = inputs.haar(8, rng, 200)
    np.testing.assert_allclose(O.gram(Qh, range(8), range(8)), np.eye(8), atol=1e-14)


def test_svd_parallel_rounds_equal_sequential():
    # disjoint pairs of a round touch disjoint columns: the parallel form
    # gives bit-identical results
    G, _ = inputs.svd_case(60, 20, 23)
    a = O.svd(G, nthreads=1)
    b = O.svd(G, nthreads=4)
    assert a.status == b.status == 0 and a.sweeps == b.sweeps
    np.testing.assert_array_equal(a.S, b.S)
    np.testing.assert_array_equal(a.U, b.U)
    np.testing.assert_array_equal(a.V, b.V)


# --------------------------------------------------------------------------
# Reduced QR (preprocessing of the one-sided SVD, §6)
# --------------------------------------------------------------------------

def test_qr_recovers_constructed_factors():
    # G = Q0 R0 with Q0 orthonormal columns and R0 upper triangular with a
    # positive diagonal: the factorization is unique, so the oracle returns them
    rng = np.random.default_rng(31)
    m, n = 90, 30
    Q0 = inputs.haar(n, rng, m)
    R0 = np.triu(rng.standard_normal((n, n)))
    R0[np.diag_indices(n)] = np.abs(R0[np.diag_indices(n)]) + 0.5
    Q, R = O.qr(Q0 @ R0)
    np.testing.assert_allclose(R, R0, atol=1e-13 * np.abs(R0).max())
    np.testing.assert_allclose(Q, Q0, atol=1e-13)
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0)


def test_qr_special_cases_and_numpy():
    rng = np.random.default_rng(32)
    # upper triangular with positive diagonal: Q = I, R = G
    T = np.triu(rng.standard_normal((12, 12))) + 3 * np.eye(12)
    Q, R = O.qr(T)
    np.testing.assert_allclose(Q, np.eye(12), atol=1e-15)
    np.testing.assert_allclose(R, T, atol=1e-14)
    # orthonormal columns: R = I
    Qh = inputs.haar(10, rng, 40)
    Q, R = O.qr(Qh)
    np.testing.assert_allclose(R, np.eye(10), atol=1e-14)
    # against LAPACK through numpy, with the signs of R's diagonal made positive
    G, _ = inputs.svd_case(200, 50, 33)
    Qn, Rn = np.linalg.qr(G)
    d = np.sign(np.diag(Rn))
    Q, R = O.qr(G)
    np.testing.assert_allclose(R, d[:, None] * Rn, atol=1e-13 * np.abs(Rn).max())
    np.testing.assert_allclose(Q, Qn * d, atol=1e-10)
    np.testing.assert_allclose(Q.T @ Q, np.eye(50), atol=1e-15 * 50)
    assert np.linalg.norm(G - Q @ R) <= 1e-15 * np.linalg.norm(G) * 10


# --------------------------------------------------------------------------
# Relative threshold (Demmel & Veselic): graded positive definite D H D
# --------------------------------------------------------------------------

dhd = inputs.graded_dhd  # A = D H D: eigenvalues graded over 10^-2span, fixed to relative accuracy


def test_relative_threshold_diagonal_is_fixed_point():
    d = 10.0 ** (-np.arange(10) * 2.0)
    r = O.eig(np.diag(d * d), relative=True)
    assert r.status == 0 and r.rotations == 0
    np.testing.assert_array_equal(r.W, np.sort(d * d))


@pytest.mark.parametrize("order", [0, 1])
def test_relative_threshold_graded_mpmath(order):
    # every eigenvalue of a graded D H D, down to 1e-22, to high relative
    # accuracy (mpmath at 60 digits as the reference)
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    n = 12
    A, _ = dhd(n, 41, 11.0)
    ref = np.sort(np.array([float(x) for x in mpmath.eigsy(mpmath.matrix(A.tolist()), eigvals_only=True)]))
    r = O.eig(A, relative=True, tol=EPS, order=order, nthreads=4 if order else 1)
    assert r.status == 0
    assert np.max(np.abs(r.W - ref) / np.abs(ref)) <= 50 * n * EPS


def test_relative_threshold_reaches_what_the_absolute_test_misses():
    # blockdiag(diag(1 .. 0.3), 1e-20 D H D): the absolute stop test sees
    # off(A) <= 1e-14 ||A||_F at once and returns the small block's diagonal
    # (relative errors of order one); the relative threshold rotates it
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    S, _ = dhd(8, 42, 2.0)
    n = 16
    A = np.zeros((n, n))
    A[:8, :8] = np.diag(np.linspace(1.0, 0.3, 8))
    A[8:, 8:] = 1e-20 * S
    ref = np.sort(np.array([float(x) for x in mpmath.eigsy(mpmath.matrix(A.tolist()), eigvals_only=True)]))
    ab = O.eig(A, tol=1e-14)
    assert ab.status == 0 and ab.sweeps == 0
    assert np.max(np.abs(ab.W - ref) / np.abs(ref)) > 1e-2
    r = O.eig(A, relative=True, tol=EPS)
    assert r.status == 0 and r.sweeps >= 2
    assert np.max(np.abs(r.W - ref) / np.abs(ref)) <= 50 * n * EPS


# --------------------------------------------------------------------------
# Pivoting step (§2.1, convergence conditions): LU with partial pivoting on
# the leading rows of V_hat selects the column permutation P
# --------------------------------------------------------------------------

def _perm_from_getrf(piv, cols):
    perm = np.arange(cols)
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    return perm


@pytest.mark.parametrize("rows,seed", [(1, 0), (3, 1), (8, 2), (32, 3), (64, 4), (64, 5)])
def test_lupp_cols_matches_lapack_getrf(rows, seed):
    # LAPACK's dgetrf on M^T: the same pivot rows (Gaussian entries: no near ties)
    import scipy.linalg as sl
    M = np.random.default_rng(seed).standard_normal((rows, 2 * rows))
    perm = O.lupp_cols(M)
    _, piv = sl.lu_factor(M.T)
    np.testing.assert_array_equal(perm, _perm_from_getrf(piv, 2 * rows))
    assert sorted(perm) == list(range(2 * rows))


def test_lupp_cols_pivots_are_final():
    # partial pivoting on the already permuted matrix swaps nothing, and every
    # multiplier of its LU factor is at most 1 in magnitude
    import scipy.linalg as sl
    M = np.random.default_rng(9).standard_normal((16, 32))
    perm = O.lupp_cols(M)
    Pm, L, U = sl.lu(M[:, perm].T)
    np.testing.assert_array_equal(Pm, np.eye(32))
    assert np.max(np.abs(L)) <= 1.0
    np.testing.assert_array_equal(O.lupp_cols(M[:, perm]), np.arange(32))


def test_lupp_cols_special_cases():
    b = 6
    Z, I = np.zeros((b, b)), np.eye(b)
    # [0 | I]: the identity half is selected, in order; the rest follows in
    # the order of the swaps
    np.testing.assert_array_equal(O.lupp_cols(np.hstack([Z, I])), list(range(b, 2 * b)) + list(range(b)))
    np.testing.assert_array_equal(O.lupp_cols(np.hstack([I, Z])), np.arange(2 * b))  # nothing to do
    np.testing.assert_array_equal(O.lupp_cols(np.zeros((b, 2 * b))), np.arange(2 * b))  # ties: first index
    # a rotation whose leading block is singular: the block swap [[0, I], [I, 0]]
    # gives V_11 = 0; the selected columns make (V P)_11 = I
    V = np.block([[Z, I], [I, Z]])
    perm = O.lupp_cols(V[:b])
    np.testing.assert_array_equal((V[:, perm])[:b, :b], I)


def test_lupp_cols_well_conditioned_leading_block():
    # rotation V_hat = blockdiag(H1, H2) [[C, -S], [S, C]] with cos/sin
    # diagonal C, S (angles near pi/2): V_11 = H1 C is nearly singular,
    # the selected columns give a leading block with sigma_min bounded away
    # from zero (here at least 1/4)
    b = 16
    rng = np.random.default_rng(11)
    H1, H2 = inputs.haar(b, rng), inputs.haar(b, rng)
    th = np.pi / 2 - 1e-9 * rng.random(b)
    C, S = np.diag(np.cos(th)), np.diag(np.sin(th))
    V = np.block([[H1 @ C, -H1 @ S], [H2 @ S, H2 @ C]])
    assert np.linalg.norm(V.T @ V - np.eye(2 * b)) < 1e-13
    assert np.linalg.svd(V[:b, :b], compute_uv=False)[-1] < 1e-8
    perm = O.lupp_cols(V[:b])
    assert np.linalg.svd(V[:b][:, perm[:b]], compute_uv=False)[-1] >= 0.25
