"""GPU parity of the blocked Jacobi eigensolver against the CPU oracle.

Every call goes through the C-ABI library (libjacobi.so) via the ctypes
binding; the oracle is the plain FP64 scalar Jacobi of oracle/ plus its
long-double checkers.  Tolerances: eigenvalues within 1e-12 of
the oracle relative to ||A||_2; ||A - Q D Q^T||_F / ||A||_F <= 1e-12 and
||Q^T Q - I||_F <= 1e-12 measured in long double.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_28952_amd import inputs

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def oracle_fixture(name):
    """Eigenvalues the oracle computed for a full-size workload
    (tests/golden/make_fullsize_oracle.py)."""
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def check_graded_bars(W, ref):
    """The bars for a graded spectrum, per eigenvalue: within 1e-12 ||A||_2 of
    the oracle; relative 1e-10 where |lambda| >= 1e-6 ||A||_2; absolute
    1e-15 ||A||_2 below that.  Returns the error profile."""
    scale = np.max(np.abs(ref))
    err = np.abs(W - ref)
    big = np.abs(ref) >= 1e-6 * scale
    prof = {"max_abs": float(err.max() / scale), "max_rel_big": float(np.max(err[big] / np.abs(ref[big]))),
            "max_abs_small": float(err[~big].max() / scale) if (~big).any() else 0.0}
    assert prof["max_abs"] <= 1e-12, prof
    assert prof["max_rel_big"] <= 1e-10, prof
    assert prof["max_abs_small"] <= 1e-15, prof
    return prof


@pytest.fixture(scope="module")
def jx():
    import torch
    from paper_2608_28952_amd import jacobi
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    jacobi.lib()
    return jacobi


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def eig_gpu(jx, A, **kw):
    uplo = kw.pop("uplo", "U")
    Q0 = kw.pop("Q0", None)
    check = kw.pop("check", True)
    o = jx.opts_default(**kw)
    W, Q, info = jx.jacobi_eig(dev(A), uplo=uplo, Q0=dev(Q0) if Q0 is not None else None, opts=o, check=check)
    return host(W), (host(Q) if Q is not None else None), info


# --------------------------------------------------------------------------
# Kernel level
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m2", [32, 64, 128])
def test_subproblem_to_convergence_matches_oracle(jx, m2):
    rng = np.random.default_rng(m2)
    mats = []
    for k in range(5):
        X = rng.standard_normal((m2, m2))
        mats.append(X + X.T)
    mats.append(np.diag(rng.standard_normal(m2)))           # already diagonal
    mats.append(np.kron(np.eye(m2 // 2), [[1.0, 1e-300], [1e-300, 1.0]]))  # tiny couplings, equal diagonal
    A = np.stack(mats)
    print(f"subproblem m2={m2}", flush=True)
    V, D = jx.jacobi_subproblem_solve(dev(A), inner_sweeps=0)
    V, D = host(V), host(D)
    for k in range(A.shape[0]):
        nrm = np.linalg.norm(A[k], 2)
        w_ora = O.eig(A[k]).W
        assert np.max(np.abs(np.sort(np.diag(D[k])) - w_ora)) <= 1e-12 * nrm
        assert np.linalg.norm(V[k].T @ V[k] - np.eye(m2)) <= 50 * m2 * EPS
        assert np.linalg.norm(V[k].T @ A[k] @ V[k] - D[k]) <= 50 * m2 * EPS * nrm
        assert O.offnorm(D[k]) <= 1e-13 * np.linalg.norm(A[k])


@pytest.mark.parametrize("m2", [32, 128])
def test_subproblem_one_sweep_is_orthogonal_similarity(jx, m2):
    rng = np.random.default_rng(7 + m2)
    X = rng.standard_normal((3, m2, m2))
    A = X + X.transpose(0, 2, 1)
    V, D = jx.jacobi_subproblem_solve(dev(A), inner_sweeps=1)
    V, D = host(V), host(D)
    for k in range(3):
        assert np.linalg.norm(V[k].T @ V[k] - np.eye(m2)) <= 50 * m2 * EPS
        assert np.linalg.norm(V[k].T @ A[k] @ V[k] - D[k]) <= 50 * m2 * EPS * np.linalg.norm(A[k])
        assert O.offnorm(D[k]) < 0.8 * O.offnorm(A[k])  # one sweep: a strict decrease
    # deterministic: identical bits on a second run
    V2, D2 = jx.jacobi_subproblem_solve(dev(A), inner_sweeps=1)
    assert np.array_equal(host(V2), V) and np.array_equal(host(D2), D)


@pytest.mark.parametrize("n,b,rnd", [(256, 64, 0), (384, 64, 2), (256, 32, 3), (512, 32, 5)])
def test_block_step_matches_oracle(jx, n, b, rnd):
    """One step of Alg. 2 on explicit data against the long-double oracle."""
    rng = np.random.default_rng(n + b)
    A, _ = inputs.eig_uniform(n, 40 + rnd)
    Q = inputs.haar(n, rng)
    N = n // b
    pairs = O.rr_list(N)[rnd]
    Vh = np.stack([inputs.haar(2 * b, rng) for _ in pairs])
    Dh = []
    for _ in pairs:
        X = rng.standard_normal((2 * b, 2 * b)) * 1e-3
        Dh.append(np.diag(rng.standard_normal(2 * b)) + X + X.T)
    Dh = np.stack(Dh)
    print(f"block step n={n} b={b}", flush=True)
    Ag, Qg = jx.jacobi_block_step(dev(A), dev(Q), b, pairs, dev(Vh), dev(Dh))
    Ar, Qr = O.block_step(A, Q, b, pairs, list(Vh), list(Dh))
    Ag, Qg = host(Ag), host(Qg)
    # FP64 GEMM bound: two products of order 2b per entry
    tolA = 8 * (2 * b) * EPS * np.max(np.abs(A)) * 4
    assert np.max(np.abs(Ag - Ar)) <= tolA
    assert np.max(np.abs(Qg - Qr)) <= 8 * (2 * b) * EPS
    assert np.array_equal(Ag, Ag.T)


def _rotation_near_singular_lead(b, rng):
    """V = blockdiag(H1, H2) [[C, -S], [S, C]] with angles near pi/2: an
    orthogonal 2b x 2b matrix whose leading b x b block is nearly singular."""
    H1, H2 = inputs.haar(b, rng), inputs.haar(b, rng)
    th = np.pi / 2 - 1e-3 * rng.random(b)
    C, S = np.diag(np.cos(th)), np.diag(np.sin(th))
    return np.block([[H1 @ C, -H1 @ S], [H2 @ S, H2 @ C]])


@pytest.mark.parametrize("n,b,rnd", [(256, 64, 0), (384, 64, 2), (256, 32, 3), (512, 32, 5)])
def test_pivot_step_matches_oracle(jx, n, b, rnd):
    """The pivoting step (LU with partial pivoting on V_hat's leading rows) in
    the solver's storage: the permutation equals the oracle's bit for bit,
    V_hat P and P^T D_hat P are exact permutations, other blocks untouched."""
    rng = np.random.default_rng(7 * n + b)
    A, _ = inputs.eig_uniform(n, 60 + rnd)
    A = np.triu(A) + np.triu(A, 1).T  # exactly symmetric
    N = n // b
    pairs = O.rr_list(N)[rnd]
    # half Haar rotations, half with a nearly singular leading block
    Vh = np.stack([inputs.haar(2 * b, rng) if k % 2 else _rotation_near_singular_lead(b, rng)
                   for k in range(len(pairs))])
    print(f"pivot step n={n} b={b}", flush=True)
    Ag, Vg, perm = jx.jacobi_pivot_step(dev(A), b, pairs, dev(Vh))
    Ag, Vg, perm = host(Ag), host(Vg), host(perm)
    Ar = A.copy()
    for k, (I, J) in enumerate(pairs):
        pk = O.lupp_cols(Vh[k][:b])
        np.testing.assert_array_equal(perm[k], pk)
        np.testing.assert_array_equal(Vg[k], Vh[k][:, pk])
        idx = np.r_[I * b:(I + 1) * b, J * b:(J + 1) * b]
        Ar[np.ix_(idx, idx)] = A[np.ix_(idx, idx)][np.ix_(pk, pk)]
        # the selected columns give a leading block far from singular
        assert np.linalg.svd(Vg[k][:b, :b], compute_uv=False)[-1] >= 1e-2
    np.testing.assert_array_equal(Ag, Ar)


@pytest.mark.parametrize("n,b,graded,prec", [(512, 32, False, 0), (1024, 64, False, 0), (1024, 64, True, 0),
                                             (1024, 64, True, 1)])
def test_eig_pivot_matches_oracle(jx, n, b, graded, prec):
    """Blocked solve with the pivoting step after every subproblem of the
    FP64 sweeps (the FP32 phase of the ladder runs without it): the same
    eigen-decomposition as the oracle, eigenvalues within 1e-12 ||A||_2."""
    A, _ = (inputs.eig_graded if graded else inputs.eig_uniform)(n, 90 + n)
    W, Q, info = eig_gpu(jx, A, block=b, pivot=1, precision=prec)
    W0, _, info0 = eig_gpu(jx, A, block=b, want_vectors=0)
    print(f"pivot n={n} b={b} graded={graded}: sweeps {info['sweeps']} (without pivoting {info0['sweeps']})",
          flush=True)
    assert info["status"] == 0, info
    _check_against_oracle(A, W, Q)
    Wv, _, infov = eig_gpu(jx, A, block=b, pivot=1, want_vectors=0)
    assert infov["status"] == 0
    assert np.max(np.abs(Wv - W)) <= 1e-12 * np.max(np.abs(W))


@pytest.mark.parametrize("n,b,rnd", [(256, 64, 0), (384, 64, 2), (256, 32, 3), (512, 32, 5)])
def test_block_step_fp32_matches_oracle(jx, n, b, rnd):
    """The FP32 kernels of the precision ladder's FP32 phase (single-block
    critical tiles split over workgroups, two-block and whole tiles, the Q
    update) against the oracle's step on the same FP32-rounded inputs."""
    rng = np.random.default_rng(n + b + 1)
    A, _ = inputs.eig_uniform(n, 50 + rnd)
    Q = inputs.haar(n, rng)
    N = n // b
    pairs = O.rr_list(N)[rnd]
    Vh = np.stack([inputs.haar(2 * b, rng) for _ in pairs])
    Dh = []
    for _ in pairs:
        X = rng.standard_normal((2 * b, 2 * b)) * 1e-3
        Dh.append(np.diag(rng.standard_normal(2 * b)) + X + X.T)
    Dh = np.stack(Dh)
    r32 = lambda M: M.astype(np.float32).astype(np.float64)
    A, Q, Vh, Dh = r32(A), r32(Q), r32(Vh), r32(Dh)
    print(f"block step fp32 n={n} b={b}", flush=True)
    Ag, Qg = jx.jacobi_block_step(dev(A), dev(Q), b, pairs, dev(Vh), dev(Dh), fp32=True)
    Ar, Qr = O.block_step(A, Q, b, pairs, list(Vh), list(Dh))
    Ag, Qg = host(Ag), host(Qg)
    # FP32 accumulation: two products of order 2b per entry, rounding of the result
    eps32 = float(np.finfo(np.float32).eps)
    assert np.max(np.abs(Ag - Ar)) <= 4 * (2 * b) * eps32 * np.max(np.abs(A))
    assert np.max(np.abs(Qg - Qr)) <= 4 * (2 * b) * eps32
    assert np.array_equal(Ag, Ag.T)
    # FP32 results: the widened values are FP32 numbers
    assert np.array_equal(r32(Ag), Ag)


def test_block_step_identity_rotation_is_exact(jx):
    n, b = 256, 64
    A, _ = inputs.eig_uniform(n, 3)
    pairs = O.rr_list(n // b)[1]
    I2 = np.stack([np.eye(2 * b)] * len(pairs))
    D = []
    for (I, J) in pairs:
        idx = np.r_[I * b:(I + 1) * b, J * b:(J + 1) * b]
        D.append(A[np.ix_(idx, idx)])
    Ag, Qg = jx.jacobi_block_step(dev(A), dev(np.eye(n)), b, pairs, dev(I2), dev(np.stack(D)))
    assert np.array_equal(host(Ag), A)
    assert np.array_equal(host(Qg), np.eye(n))


# --------------------------------------------------------------------------
# Full solver against the oracle
# --------------------------------------------------------------------------

def _check_against_oracle(A, W, Q, tol_eig=1e-12, ora_tol=1e-14):
    # the oracle's round-robin rounds, in parallel over a round's disjoint
    # rotations for the larger orders
    ora = O.eig(A, tol=ora_tol, order=1, nthreads=1 if A.shape[0] < 256 else min(16, os.cpu_count() or 1))
    assert ora.status == 0
    nrm = max(np.max(np.abs(ora.W)), 1e-300)
    assert np.max(np.abs(W - ora.W)) <= tol_eig * nrm, np.max(np.abs(W - ora.W)) / nrm
    if Q is not None:
        res, orth, _, _ = O.check_eig(A, W, Q)
        assert res <= 1e-12 and orth <= 1e-12, (res, orth)


@pytest.mark.parametrize("n", [2, 3, 17, 64, 100, 128, 130, 200])
def test_eig_small_parity(jx, n):
    A, _ = inputs.eig_uniform(n, 1000 + n)
    print(f"eig n={n}", flush=True)
    W, Q, info = eig_gpu(jx, A)
    assert info["status"] == 0
    _check_against_oracle(A, W, Q)


@pytest.mark.parametrize("n", [2, 3, 17, 64, 129, 255])
def test_eig_scalar_b1_matches_oracle(jx, n):
    """b = 1: scalar two-sided Jacobi in round-robin rounds (Alg. 1 with
    b = 1), odd orders with a placeholder index."""
    A, _ = inputs.eig_uniform(n, 300 + n)
    W, Q, info = eig_gpu(jx, A, block=1)
    assert info["status"] == 0, info
    _check_against_oracle(A, W, Q)
    Wv, Qv, _ = eig_gpu(jx, A, block=1, want_vectors=0)
    assert Qv is None and np.max(np.abs(Wv - W)) <= 1e-14 * np.max(np.abs(W))


def test_eig_scalar_b1_config_n256(jx):
    """The scalar workload: n = 256, Haar Q, lambda ~ U[-1, 1], seed 1, round-robin
    rounds of 128 rotations, stop at off(A) <= 1e-14 ||A||_F."""
    A, lam = inputs.eig_uniform(256, 1)
    W, Q, info = eig_gpu(jx, A, block=1)
    print(f"scalar n=256: sweeps {info['sweeps']}, off_rel {info['off_rel']:.2e}", flush=True)
    assert info["status"] == 0 and info["off_rel"] <= 1e-14
    _check_against_oracle(A, W, Q)
    assert np.max(np.abs(W - np.sort(lam))) <= 256 * EPS


@pytest.mark.parametrize("n,span", [(12, 11.0), (64, 10.0), (200, 6.0)])
def test_eig_scalar_relative_threshold_graded(jx, n, span):
    """b = 1 with the relative threshold on a graded positive definite D H D:
    every eigenvalue, down to 10^-2span, to high relative accuracy, the same
    as the oracle's relative mode (each side within 50 n u of the exact
    values, which the entries fix to that accuracy)."""
    A, _ = inputs.graded_dhd(n, 41 + n, span)
    print(f"relative threshold n={n} span={span}", flush=True)
    W, Q, info = eig_gpu(jx, A, block=1, threshold=1, tol=EPS)
    assert info["status"] == 0, info
    ora = O.eig(A, relative=True, tol=EPS, order=1, nthreads=4)
    assert ora.status == 0
    assert np.max(np.abs(W - ora.W) / np.abs(ora.W)) <= 100 * n * EPS
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13 * n


def test_eig_scalar_relative_threshold_small_block(jx):
    """blockdiag(diag(1 .. 0.3), 1e-20 D H D): the absolute stop test is met
    before any rotation and returns the tiny block's diagonal; the relative
    threshold rotates it and matches the oracle's relative mode."""
    S, _ = inputs.graded_dhd(8, 42, 2.0)
    A = np.zeros((16, 16), order="F")
    A[:8, :8] = np.diag(np.linspace(1.0, 0.3, 8))
    A[8:, 8:] = 1e-20 * S
    ora = O.eig(A, relative=True, tol=EPS)
    Wa, _, ia = eig_gpu(jx, A, block=1, tol=1e-14)
    assert ia["status"] == 0 and ia["sweeps"] == 0
    assert np.max(np.abs(Wa - ora.W) / np.abs(ora.W)) > 1e-2
    W, _, info = eig_gpu(jx, A, block=1, threshold=1, tol=EPS)
    assert info["status"] == 0 and info["sweeps"] >= 2
    assert np.max(np.abs(W - ora.W) / np.abs(ora.W)) <= 100 * 16 * EPS


def test_eig_config_n256_uniform(jx):
    """n = 256, Haar Q, lambda ~ U[-1, 1], seed 1, tol 1e-14."""
    A, lam = inputs.eig_uniform(256, 1)
    W, Q, info = eig_gpu(jx, A)
    assert info["status"] == 0 and info["off_rel"] <= 1e-14
    _check_against_oracle(A, W, Q)
    assert np.max(np.abs(W - np.sort(lam))) <= 256 * EPS


@pytest.mark.parametrize("b,order,uplo", [(32, 0, "U"), (64, 0, "L"), (32, 1, "L"), (64, 1, "U"), (32, 2, "U"),
                                           (64, 2, "L")])
def test_eig_blocks_orderings_triangles(jx, b, order, uplo):
    n = 320
    A, _ = inputs.eig_normal(n, 77)
    Ain = A.copy()
    # poison the unused triangle: the solver must not read it
    if uplo == "U":
        Ain[np.tril_indices(n, -1)] = np.nan
    else:
        Ain[np.triu_indices(n, 1)] = np.nan
    W, Q, info = eig_gpu(jx, Ain, block=b, ordering=order, uplo=uplo)
    assert info["status"] == 0
    _check_against_oracle(A, W, Q)


@pytest.mark.parametrize("n,kind,prec,vec", [(200, "graded", 0, 1), (640, "graded", 0, 1), (1024, "graded", 0, 0),
                                             (512, "uniform", 1, 1), (1000, "graded", 1, 1)])
def test_eig_sorted_ordering_matches_oracle(jx, n, kind, prec, vec):
    """Round-robin with the indices re-sorted by the diagonal before each
    sweep: an exact permutation, so the results meet the same bars against
    the oracle (FP64 and the FP32 ladder, with and without vectors)."""
    gen = {"uniform": inputs.eig_uniform, "graded": inputs.eig_graded}[kind]
    A, _ = gen(n, 90 + n)
    print(f"eig sorted n={n} {kind} prec={prec} vectors={vec}", flush=True)
    W, Q, info = eig_gpu(jx, A, ordering=2, precision=prec, want_vectors=vec)
    assert info["status"] == 0, info
    if vec:
        _check_against_oracle(A, W, Q)
    else:
        ora = O.eig(A, order=1, nthreads=min(16, os.cpu_count() or 1), want_vectors=False)
        assert np.max(np.abs(W - ora.W)) <= 1e-12 * np.max(np.abs(ora.W))


def test_eig_sorted_ordering_takes_fewer_sweeps(jx):
    """On a graded spectrum the re-sorted ordering converges in fewer sweeps
    than the static round-robin (measured: see the printed counts)."""
    A, _ = inputs.eig_graded(1024, 2)
    _, _, i0 = eig_gpu(jx, A, ordering=0, block=64)
    _, _, i2 = eig_gpu(jx, A, ordering=2, block=64)
    print(f"n=1024 graded sweeps: round-robin {i0['sweeps']}, sorted {i2['sweeps']}", flush=True)
    assert i0["status"] == 0 and i2["status"] == 0
    assert i2["sweeps"] < i0["sweeps"]


def test_eig_antidiag_four_blocks(jx):
    """Alg. 3's groups on N = 4 blocks: a placeholder pair of round r + 2 is a
    rotated pair of round r, so its block reaches the next round's critical
    kernel through the copy made after round r (not through a tile)."""
    n = 256
    A, _ = inputs.eig_normal(n, 81)
    print("eig n=256 b=64 antidiag", flush=True)
    W, Q, info = eig_gpu(jx, A, block=64, ordering=1)
    assert info["status"] == 0
    _check_against_oracle(A, W, Q)


def test_eig_graded_512_relative_accuracy(jx):
    """Graded spectrum lambda_i = +-10^(-8 i / n): absolute 1e-12 and per-eigenvalue
    relative 1e-10 for |lambda| >= 1e-6 ||A||_2 against the oracle."""
    n = 512
    A, lam = inputs.eig_graded(n, 2)
    W, Q, info = eig_gpu(jx, A)
    assert info["status"] == 0
    ora = O.eig(A, order=1)
    big = np.abs(ora.W) >= 1e-6
    assert np.max(np.abs(W - ora.W)) <= 1e-12
    assert np.max(np.abs(W - ora.W)[big] / np.abs(ora.W[big])) <= 1e-10
    assert np.max(np.abs(W - ora.W)[~big]) <= 1e-15
    res, orth, _, _ = O.check_eig(A, W, Q)
    assert res <= 1e-12 and orth <= 1e-12


def test_eig_sweep_cap_with_refinement(jx):
    """opts.max_sweeps bounds the sweeps to convergence also when the
    orthogonality refinement runs inside the quadratic phase: one sweep
    short of what the full solve needs, the solve stops at the cap with
    status 1 (not converged) instead of refining and sweeping on."""
    n = 1024
    A, lam = inputs.eig_graded(n, 11)
    W, _, info = eig_gpu(jx, A, block=64)
    assert info["status"] == 0, info
    S = info["sweeps"]
    print(f"graded n={n} b=64: {S} sweeps", flush=True)
    assert np.max(np.abs(W - np.sort(lam))) <= 1e-12 * np.max(np.abs(lam))
    for cap in (S - 1, S - 2):
        _, _, ic = eig_gpu(jx, A, block=64, max_sweeps=cap, check=False)
        assert ic["status"] == 1 and ic["sweeps"] == cap, (cap, ic)


def test_eig_values_only_and_unsorted(jx):
    A, _ = inputs.eig_uniform(150, 5)
    Wv, Qv, info = eig_gpu(jx, A, want_vectors=0)
    assert Qv is None and info["status"] == 0
    Wf, Qf, _ = eig_gpu(jx, A)
    assert np.max(np.abs(Wv - Wf)) <= 1e-13
    Wu, Qu, _ = eig_gpu(jx, A, sort=0)
    assert np.max(np.abs(np.sort(Wu) - Wf)) <= 1e-13
    res, orth, _, _ = O.check_eig(A, Wu, Qu)
    assert res <= 1e-12 and orth <= 1e-12


def test_eig_inner_to_convergence_same_answer(jx):
    A, _ = inputs.eig_uniform(256, 9)
    W1, Q1, i1 = eig_gpu(jx, A, inner_max_sweeps=1)
    W0, Q0, i0 = eig_gpu(jx, A, inner_max_sweeps=0)
    assert i0["status"] == 0 and i1["status"] == 0
    assert np.max(np.abs(W1 - W0)) <= 1e-13


def test_eig_warm_start_resume(jx):
    A, _ = inputs.eig_uniform(256, 13)
    W2, Q2, i2 = eig_gpu(jx, A, max_sweeps=2, refine=0, check=False)
    assert i2["status"] == 1
    W, Q, info = eig_gpu(jx, A, Q0=Q2)
    assert info["status"] == 0
    Wf, _, inf_full = eig_gpu(jx, A)
    assert np.max(np.abs(W - Wf)) <= 1e-13
    assert info["sweeps"] < inf_full["sweeps"]
    _check_against_oracle(A, W, Q)


def test_eig_edge_cases(jx):
    import torch
    # n = 1
    W, Q, info = eig_gpu(jx, np.array([[3.5]]))
    assert W[0] == 3.5 and Q[0, 0] == 1.0 and info["status"] == 0
    # n = 0
    W, Q, info = jx.jacobi_eig(torch.zeros((0, 0), dtype=torch.float64, device="cuda"))
    assert W.numel() == 0 and info["status"] == 0
    # diagonal input: no rotation at all, Q a permutation
    d = np.array([3.0, -1.0, 2.0, 0.5, -7.0, 4.0])
    W, Q, info = eig_gpu(jx, np.diag(d))
    assert np.array_equal(W, np.sort(d)) and info["sweeps"] == 0
    assert np.array_equal(np.abs(Q), np.eye(6)[:, np.argsort(d)])
    # non-finite input
    A, _ = inputs.eig_uniform(64, 2)
    A[5, 9] = A[9, 5] = np.inf
    _, _, info = eig_gpu(jx, A, check=False)
    assert info["status"] == 2
    # not converged
    A, _ = inputs.eig_uniform(300, 2)
    _, _, info = eig_gpu(jx, A, max_sweeps=1, check=False)
    assert info["status"] == 1 and info["sweeps"] == 1


@pytest.mark.parametrize("block", [0, 1])
def test_eig_degenerate_spectra(jx, block):
    """Zero and identity matrices (every pair skipped: no sweep, W and Q
    exact), and three clusters of exactly equal eigenvalues: A = H diag(lam)
    H^T / 256 with H the Sylvester-Hadamard matrix of order 256 and lam in
    {-1, 1/4, 2} is exact in FP64, so its spectrum is exactly lam (the
    vectors of a cluster are not unique: eigenvalues against lam, residual
    and orthogonality in long double)."""
    import scipy.linalg as sl
    n = 256
    for A, lam in ((np.zeros((n, n)), 0.0), (np.eye(n), 1.0)):
        W, Q, info = eig_gpu(jx, A, block=block)
        assert info["status"] == 0 and info["sweeps"] == 0
        assert np.all(W == lam) and np.array_equal(Q, np.eye(n))
    H = sl.hadamard(n).astype(np.float64)
    lam = np.repeat([-1.0, 0.25, 2.0], [80, 96, 80])[np.random.default_rng(3).permutation(n)]
    A = np.asfortranarray((H * lam) @ H.T / n)
    assert np.array_equal(A, A.T)
    W, Q, info = eig_gpu(jx, A, block=block)
    print(f"clusters block={block}: sweeps {info['sweeps']} status {info['status']}", flush=True)
    assert info["status"] == 0
    assert np.max(np.abs(W - np.sort(lam))) <= 1e-12 * 2.0
    res, orth, _, _ = O.check_eig(A, W, Q)
    assert res <= 1e-12 and orth <= 1e-12, (res, orth)


def test_eig_scalar_b1_largest_order(jx):
    """b = 1 at its largest order, n = 1024 (one launch per round over 512
    workgroups), against the oracle."""
    A, _ = inputs.eig_uniform(1024, 55)
    W, Q, info = eig_gpu(jx, A, block=1)
    print(f"scalar n=1024: sweeps {info['sweeps']}", flush=True)
    assert info["status"] == 0
    _check_against_oracle(A, W, Q)


def test_eig_workspace_too_small(jx):
    import torch
    A, _ = inputs.eig_uniform(200, 1)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    W, Q, info = jx.jacobi_eig(dev(A), work=small, check=False)
    assert info["status"] == -100
    need = jx.jacobi_eig_workspace(200)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    W, Q, info = jx.jacobi_eig(dev(A), work=work)
    assert info["status"] == 0
    _check_against_oracle(A, host(W), host(Q))


def test_eig_deterministic(jx):
    A, _ = inputs.eig_uniform(384, 21)
    W1, Q1, _ = eig_gpu(jx, A)
    W2, Q2, _ = eig_gpu(jx, A)
    assert np.array_equal(W1, W2) and np.array_equal(Q1, Q2)


def test_eig_metamorphic(jx):
    A, _ = inputs.eig_uniform(192, 31)
    W, _, _ = eig_gpu(jx, A)
    Ws, _, _ = eig_gpu(jx, A + 3.0 * np.eye(192))
    Wn, _, _ = eig_gpu(jx, -A)
    assert np.max(np.abs(Ws - (W + 3.0))) <= 1e-12 * 4
    assert np.max(np.abs(Wn + W[::-1])) <= 1e-12


# --------------------------------------------------------------------------
# Full size: n = 4096, b = 64, graded spectrum (the benchmark workload)
# --------------------------------------------------------------------------

def test_eig_n4096_graded_full_size(jx):
    """The benchmark workload against the oracle's eigenvalues of the same
    matrix (fixture), element by element under the graded-spectrum bars, and
    the full long-double residual and orthogonality."""
    n = 4096
    A, lam = inputs.eig_graded(n, 2)
    print("eig n=4096 graded", flush=True)
    W, Q, info = eig_gpu(jx, A)
    assert info["status"] == 0, info
    prof = check_graded_bars(W, oracle_fixture("eig_graded_n4096_seed2.txt"))
    res, orth, _, _ = O.check_eig(A, W, Q)
    print(f"  vs oracle {prof}; residual {res:.2e} orthogonality {orth:.2e}", flush=True)
    assert res <= 1e-12 and orth <= 1e-12, (res, orth)


def test_eig_n2048_b64_sixteen_pairs_per_round(jx):
    """b = 64 at n = 2048: 32 block columns, 16 pairs per round (the
    subproblem kernel at 2b = 128 and the split tile update with its partial
    last round of the persistent kernel), against the oracle's eigenvalues
    of the same matrix (fixture) and the full long-double checks."""
    n = 2048
    A, _ = inputs.eig_uniform(n, 7)
    print("eig n=2048 b=64", flush=True)
    W, Q, info = eig_gpu(jx, A, block=64)
    assert info["status"] == 0, info
    ref = oracle_fixture("eig_uniform_n2048_seed7.txt")
    assert np.max(np.abs(W - ref)) <= 1e-12 * np.max(np.abs(ref))
    res, orth, _, _ = O.check_eig(A, W, Q)
    print(f"  sweeps {info['sweeps']}, max |dW| {np.max(np.abs(W - ref)):.2e}, residual {res:.2e}, "
          f"orthogonality {orth:.2e}", flush=True)
    assert res <= 1e-12 and orth <= 1e-12, (res, orth)


# --------------------------------------------------------------------------
# Precision ladder: FP32 sweeps (FP64 subproblems), FP64 recomputation, FP64 sweeps
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,kind,b", [(320, "uniform", 32), (512, "graded", 64), (384, "normal", 64)])
def test_eig_mixed_fp32_matches_oracle(jx, n, kind, b):
    gen = {"uniform": inputs.eig_uniform, "graded": inputs.eig_graded, "normal": inputs.eig_normal}[kind]
    A, lam = gen(n, 60 + n)
    W, Q, info = eig_gpu(jx, A, precision=jx.PREC_MIXED_FP32, block=b)
    assert info["status"] == 0, info
    assert info["sweeps_by_prec"][1] > 0 and info["sweeps_by_prec"][2] > 0
    print(f"mixed n={n} {kind}: fp32 sweeps {info['sweeps_by_prec'][1]}, fp64 sweeps {info['sweeps_by_prec'][2]}")
    _check_against_oracle(A, W, Q)
    if kind == "graded":
        ora = O.eig(A, order=1)
        big = np.abs(ora.W) >= 1e-6
        assert np.max(np.abs(W - ora.W)[big] / np.abs(ora.W[big])) <= 1e-10


def test_eig_mixed_values_only(jx):
    A, _ = inputs.eig_uniform(256, 4)
    W, Q, info = eig_gpu(jx, A, precision=jx.PREC_MIXED_FP32, want_vectors=0)
    assert Q is None and info["status"] == 0
    assert np.max(np.abs(W - O.eig(A).W)) <= 1e-12


def test_eig_n4096_graded_mixed_fp32(jx):
    n = 4096
    A, lam = inputs.eig_graded(n, 2)
    W, Q, info = eig_gpu(jx, A, precision=jx.PREC_MIXED_FP32)
    assert info["status"] == 0, info
    ref = np.sort(lam)
    err = np.abs(W - ref)
    big = np.abs(ref) >= 1e-6
    print(f"mixed n=4096: sweeps {info['sweeps_by_prec']}, max abs err {err.max():.2e}, "
          f"max rel err (|lam|>=1e-6) {np.max(err[big] / np.abs(ref[big])):.2e}")
    assert err.max() <= 1e-12 and np.max(err[big] / np.abs(ref[big])) <= 1e-10
    # the FP32 phase ends where its sweeps stop halving the off-norm: as many
    # sweeps in all as plain FP64 (27); running it on to 1e-5 took 30
    assert sum(info["sweeps_by_prec"]) <= 28, info
    check_graded_bars(W, oracle_fixture("eig_graded_n4096_seed2.txt"))
    res, orth, _, _ = O.check_eig(A, W, Q)
    assert res <= 1e-12 and orth <= 1e-12, (res, orth)


def test_handoff_wait_bound_reports_nonfinite(tmp_path):
    """At 2b = 128 the subproblem kernel hands each round's rotations from the
    sweeping wave to the wave that accumulates V, through waits that are
    bounded.  A wait whose bound runs out poisons the kernel's output with NaN,
    so the solve reports a non-finite iterate (status 2) instead of returning
    wrong numbers.  A bound of one poll (JACOBI_HANDOFF_SPIN=1, read once per
    process, hence the child process) forces that path; every kernel still
    exits normally."""
    import os
    import subprocess
    import sys
    script = tmp_path / "bound.py"
    script.write_text(
        "import sys\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.dirname(os.path.abspath(__file__)))!r})\n"
        "import numpy as np, torch\n"
        "from paper_2608_28952_amd import inputs, jacobi as jx\n"
        "A, _ = inputs.eig_uniform(256, 5)\n"
        "W, Q, info = jx.jacobi_eig(torch.from_numpy(A).cuda(), opts=jx.opts_default(block=64), check=False)\n"
        "print('status', info['status'], flush=True)\n")
    env = dict(os.environ, JACOBI_HANDOFF_SPIN="1")
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "status 2" in r.stdout, r.stdout
