"""GPU parity of the batched solver (jacobi_eig_batched) against the CPU oracle.

Every matrix of a batch is checked against the scalar FP64 oracle run on the
same stored input (the FP32 matrix upcast to FP64 for FP32 batches): the
eigenvalues within 1e-12 max|lambda|, and in long double
||A - Q diag(W) Q^T||_F / ||A||_F <= 1e-12 and ||Q^T Q - I||_F <= 1e-12.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_28952_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def jx():
    import torch
    from paper_2608_28952_amd import jacobi
    assert torch.cuda.is_available()
    jacobi.lib()
    return jacobi


def pack(mats, dtype):
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    offs = np.zeros(len(mats) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)
    packed = np.empty(int(offs[-1]), dtype=dtype)
    for k, m in enumerate(mats):
        packed[offs[k]:offs[k + 1]] = np.asarray(m, dtype=np.float64).reshape(-1, order="F").astype(dtype)
    return sizes, offs, packed


def unpack(sizes, offs, W, Q):
    Ws, Qs, w = [], [], 0
    for k, n in enumerate(sizes):
        n = int(n)
        Ws.append(W[w:w + n])
        w += n
        Qs.append(Q[offs[k]:offs[k] + n * n].reshape((n, n), order="F") if Q is not None else None)
    return Ws, Qs


def run(jx, sizes, offs, packed, Q0=None, work=True, **kw):
    import torch
    o = jx.opts_default(**kw)
    dA = torch.from_numpy(packed).cuda()
    q0 = torch.from_numpy(Q0).cuda() if Q0 is not None else None
    ws = None
    if work:
        ws = torch.empty(jx.batched_workspace(sizes, packed.dtype == np.float64, o), dtype=torch.uint8, device="cuda")
    W, Q, infos = jx.jacobi_eig_batched(sizes, offs, dA, Q0=q0, opts=o, work=ws, check=False)
    Wn = W.cpu().numpy()
    Qn = Q.cpu().numpy() if kw.get("want_vectors", 1) else None
    return unpack(sizes, offs, Wn, Qn), infos


def check_against_oracle(A, w, q, tol=1e-12):
    A = np.asarray(A, dtype=np.float64)
    ora = O.eig(A)
    scale = max(np.max(np.abs(ora.W)), 1e-300)
    assert np.max(np.abs(w - ora.W)) <= tol * scale, np.max(np.abs(w - ora.W)) / scale
    if q is not None:
        res, orth, _, _ = O.check_eig(A, w, q)
        assert res <= tol and orth <= tol, (res, orth)


EDGE_SIZES = [1, 2, 3, 8, 15, 16, 17, 31, 32, 33, 47, 64, 65, 96, 127, 128, 129, 160, 192, 193, 224, 255, 256]


def edge_batch(seed, dtype):
    rng = np.random.default_rng(seed)
    mats = []
    for n in EDGE_SIZES:
        Q = inputs.haar(n, rng)
        lam = rng.standard_normal(n)
        mats.append(inputs.sym_with_spectrum(lam, Q))
    sizes, offs, packed = pack(mats, dtype)
    stored = [packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
              for k, n in enumerate(sizes)]
    return sizes, offs, packed, stored


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_edge_sizes_match_oracle(jx, dtype, precision):
    sizes, offs, packed, stored = edge_batch(11, dtype)
    prec = jx.PREC_MIXED_FP32 if precision == "mixed" else jx.PREC_FP64
    print(f"batched edge sizes dtype={np.dtype(dtype).name} precision={precision}", flush=True)
    (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=prec)
    for k, n in enumerate(sizes):
        assert infos[k]["status"] == 0, (n, infos[k])
        if precision == "fp64":
            assert infos[k]["sweeps_by_prec"][1] == 0
        check_against_oracle(stored[k], Ws[k], Qs[k])
        assert np.all(np.diff(Ws[k]) >= 0)


@pytest.mark.parametrize("block", [8, 16])
def test_batched_forced_block_sizes(jx, block):
    sizes, offs, packed = inputs.batched_case(24, 4)
    print(f"batched block={block}", flush=True)
    (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32, block=block)
    for k, n in enumerate(sizes):
        n = int(n)
        assert infos[k]["status"] == 0
        A = packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
        check_against_oracle(A, Ws[k], Qs[k])


def test_batched_equals_single_matrix_solver(jx):
    import torch
    sizes, offs, packed = inputs.batched_case(6, 9)
    (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32)
    for k, n in enumerate(sizes):
        n = int(n)
        A = packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
        W1, Q1, info1 = jx.jacobi_eig(torch.from_numpy(np.ascontiguousarray(A)).cuda())
        w1 = W1.cpu().numpy()
        assert np.max(np.abs(Ws[k] - w1)) <= 1e-12 * np.max(np.abs(w1))


def test_batched_values_only_nonfinite_and_empty(jx):
    rng = np.random.default_rng(3)
    mats = [inputs.sym_with_spectrum(rng.standard_normal(n), inputs.haar(n, rng)) for n in (20, 40, 70)]
    bad = mats[1].copy()
    bad[3, 5] = bad[5, 3] = np.nan
    mats_bad = [mats[0], bad, mats[2]]
    sizes, offs, packed = pack(mats_bad, np.float64)
    (Ws, _), infos = run(jx, sizes, offs, packed, want_vectors=0)
    assert [i["status"] for i in infos] == [0, 2, 0]
    assert np.all(np.isnan(Ws[1]))
    check_against_oracle(mats[0], Ws[0], None)
    check_against_oracle(mats[2], Ws[2], None)
    # an order-0 entry is skipped
    sizes0 = np.array([0, 20], dtype=np.int32)
    offs0 = np.array([0, 0, 400], dtype=np.int64)
    packed0 = np.asarray(mats[0], dtype=np.float64).reshape(-1, order="F").copy()
    (Ws0, Qs0), infos0 = run(jx, sizes0, offs0, packed0)
    assert infos0[0]["status"] == 0 and len(Ws0[0]) == 0
    check_against_oracle(mats[0], Ws0[1], Qs0[1])


def test_batched_graph_cache_and_determinism(jx):
    import torch
    sizes, offs, packed = inputs.batched_case(40, 21)
    o = jx.opts_default(precision=jx.PREC_MIXED_FP32)
    dA = torch.from_numpy(packed).cuda()
    ws = torch.empty(jx.batched_workspace(sizes, False, o), dtype=torch.uint8, device="cuda")
    W = torch.empty(int(sizes.sum()), dtype=torch.float64, device="cuda")
    Q = torch.empty(int(offs[len(sizes)]), dtype=torch.float64, device="cuda")
    h0, b0 = jx.batched_graph_stats()
    jx.jacobi_eig_batched(sizes, offs, dA, opts=o, work=ws, out=(W, Q))
    W1, Q1 = W.clone(), Q.clone()
    h1, b1 = jx.batched_graph_stats()
    # three replays, with eager work on the same buffers and synchronisations
    # between them: every replay equals the first call
    for rep in range(3):
        W.fill_(float(rep + 1))
        Q.fill_(-float(rep + 1))
        ws.fill_(0xA5)
        torch.cuda.synchronize()
        _, _, infos = jx.jacobi_eig_batched(sizes, offs, dA, opts=o, work=ws, out=(W, Q))
        torch.cuda.synchronize()
        assert all(i["status"] == 0 for i in infos)
        assert torch.equal(W1, W) and torch.equal(Q1, Q), rep
    h2, b2 = jx.batched_graph_stats()
    assert b1 == b0 + 1 and b2 == b1            # built once
    assert h2 == h1 + 3                          # then replayed


def test_batched_warm_start_and_fallback(jx):
    rng = np.random.default_rng(17)
    n = 64
    mats, good, badq = [], [], []
    for k in range(6):
        A = inputs.sym_with_spectrum(rng.standard_normal(n), inputs.haar(n, rng))
        mats.append(A)
        ora = O.eig(A)
        # a small rotation away from the exact eigenvectors
        S = rng.standard_normal((n, n)) * 1e-3
        S = S - S.T
        good.append(ora.Q @ O.cayley(S))
        badq.append(inputs.haar(n, rng))
    sizes, offs, packed = pack(mats, np.float64)
    q_good = np.concatenate([q.reshape(-1, order="F") for q in good])
    q_bad = np.concatenate([q.reshape(-1, order="F") for q in badq])
    (Wc, Qc), ic = run(jx, sizes, offs, packed, precision=jx.PREC_FP64)
    (Wg, Qg), ig = run(jx, sizes, offs, packed, Q0=q_good, precision=jx.PREC_FP64)
    (Wb, Qb), ib = run(jx, sizes, offs, packed, Q0=q_bad, precision=jx.PREC_FP64)
    for k in range(len(mats)):
        assert ig[k]["status"] == 0 and ig[k]["fallback_used"] == 0
        assert ig[k]["sweeps"] < ic[k]["sweeps"], (ig[k], ic[k])
        check_against_oracle(mats[k], Wg[k], Qg[k])
        assert ib[k]["status"] == 0
        check_against_oracle(mats[k], Wb[k], Qb[k])
    assert sum(i["fallback_used"] for i in ib) >= 1


def test_batched_fp32_quality_warm_start_values_only(jx):
    """A warm start orthogonal only to FP32 accuracy (exact eigenvectors
    rotated slightly, then rounded to FP32) with eigenvalues only: the
    Newton-Schulz steps must restore FP64 orthogonality before Q0^T A Q0,
    or the eigenvalues miss the 1e-12 bar."""
    rng = np.random.default_rng(19)
    mats, starts = [], []
    for n in (40, 96, 200, 256):
        A = inputs.sym_with_spectrum(rng.standard_normal(n), inputs.haar(n, rng))
        mats.append(A)
        S = rng.standard_normal((n, n)) * 1e-4
        q = O.eig(A).Q @ O.cayley(S - S.T)
        starts.append(q.astype(np.float32).astype(np.float64))
        assert np.linalg.norm(starts[-1].T @ starts[-1] - np.eye(n)) > 1e-7  # not FP64-orthogonal
    sizes, offs, packed = pack(mats, np.float64)
    q0 = np.concatenate([q.reshape(-1, order="F") for q in starts])
    (Ws, _), infos = run(jx, sizes, offs, packed, Q0=q0, precision=jx.PREC_FP64, want_vectors=0)
    for k in range(len(mats)):
        assert infos[k]["status"] == 0 and infos[k]["fallback_used"] == 0, infos[k]
        check_against_oracle(mats[k], Ws[k], None)


def test_batched_library_workspace(jx):
    sizes, offs, packed = inputs.batched_case(10, 5)
    (Ws, Qs), infos = run(jx, sizes, offs, packed, work=False, precision=jx.PREC_MIXED_FP32)
    for k, n in enumerate(sizes):
        n = int(n)
        assert infos[k]["status"] == 0
        A = packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
        check_against_oracle(A, Ws[k], Qs[k])


def test_batched_autotune_cache(jx, tmp_path):
    path = tmp_path / "tune.json"
    jx.batched_autotune(path, dtype_f64=False, per_bucket=6, seed=2)
    doc = json.loads(path.read_text())
    assert len(doc["f32_bs"]) == 5 and all(b in (8, 16) for b in doc["f32_bs"])
    assert all(m in (0, 1, 2) for m in doc["f32_mixed"])
    assert len(doc["calibration_ms"]) == 5 * 6 and all(t > 0 for t in doc["calibration_ms"])
    assert jx.batched_tuning(False, 4)[2] is True
    # a corrupt cache file gives the defaults
    bad = tmp_path / "bad.json"
    bad.write_text("{ not json")
    os.environ["JACOBI_TUNE_FILE"] = str(bad)
    try:
        assert jx.batched_tuning(False, 0)[2] is False
        sizes, offs, packed = inputs.batched_case(5, 6)
        (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32)
        assert all(i["status"] == 0 for i in infos)
        os.environ["JACOBI_TUNE_FILE"] = str(path)
        assert jx.batched_tuning(False, 4)[2] is True
    finally:
        del os.environ["JACOBI_TUNE_FILE"]


def test_batched_early_switch_level_matches_oracle(jx, tmp_path):
    """A table whose every bucket ends the FP32 phase at 1e-3 ||A||_F (mixed
    level 2): fewer FP32 sweeps, and the same results to the 1e-12 bar."""
    path = tmp_path / "tune.json"
    jx.batched_autotune(path, dtype_f64=False, per_bucket=4, seed=3)
    doc = json.loads(path.read_text())
    doc["f32_mixed"] = [2] * 5
    lvl2 = tmp_path / "level2.json"
    lvl2.write_text(json.dumps(doc))
    sizes, offs, packed = inputs.batched_case(40, 9)
    os.environ["JACOBI_TUNE_FILE"] = str(lvl2)
    try:
        assert jx.batched_tuning(False, 2)[1] == 2
        (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32)
    finally:
        del os.environ["JACOBI_TUNE_FILE"]
    (_, _), infos1 = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32)
    f32_2 = sum(i["sweeps_by_prec"][1] for i in infos)
    f32_1 = sum(i["sweeps_by_prec"][1] for i in infos1)
    print(f"FP32 sweeps: level 2 {f32_2}, level 1 {f32_1}", flush=True)
    assert f32_2 < f32_1
    for k, n in enumerate(sizes):
        n = int(n)
        assert infos[k]["status"] == 0
        A = packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
        check_against_oracle(A, Ws[k], Qs[k])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batched_degenerate_matrices(jx, precision):
    """Zero and identity matrices (no sweep, exact results) and exactly
    clustered spectra, A = H diag(lam) H^T / n with H Hadamard and lam in
    {-1, 1/4, 2} (exact in FP64): every matrix converges, eigenvalues
    within 1e-12 max|lam| of lam."""
    import scipy.linalg as sl
    mats = []
    for n in (16, 64, 128):
        H = sl.hadamard(n).astype(np.float64)
        lam = np.repeat([-1.0, 0.25, 2.0], [n * 5 // 16, n * 6 // 16, n - n * 5 // 16 - n * 6 // 16])
        lam = lam[np.random.default_rng(n).permutation(n)]
        mats += [((H * lam) @ H.T / n, np.sort(lam)), (np.zeros((n, n)), np.zeros(n)), (np.eye(n), np.ones(n))]
    sizes = np.array([A.shape[0] for A, _ in mats], dtype=np.int32)
    offs = np.zeros(len(mats) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)
    packed = np.concatenate([A.reshape(-1, order="F") for A, _ in mats])
    prec = jx.PREC_MIXED_FP32 if precision == "mixed" else jx.PREC_FP64
    (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=prec)
    for k, (A, lam) in enumerate(mats):
        assert infos[k]["status"] == 0, (k, infos[k])
        assert np.max(np.abs(Ws[k] - lam)) <= 1e-12 * 2.0
        if k % 3:  # zero and identity: nothing to rotate
            assert infos[k]["sweeps"] == 0 and np.array_equal(Qs[k], np.eye(A.shape[0]))
        else:
            res, orth, _, _ = O.check_eig(A, Ws[k], Qs[k])
            assert res <= 1e-12 and orth <= 1e-12, (k, res, orth)


def test_batched_full_workload_sampled(jx):
    """The full batched workload: 10,000 matrices, n uniform in [16, 256],
    lambda ~ N(0, 1), stored FP32, seed 4; every matrix converged, 24 sampled
    matrices checked against the oracle."""
    sizes, offs, packed = inputs.batched_case(10000, 4)
    print("batched full 10000", flush=True)
    (Ws, Qs), infos = run(jx, sizes, offs, packed, precision=jx.PREC_MIXED_FP32)
    st = np.array([i["status"] for i in infos])
    assert np.all(st == 0), np.unique(st, return_counts=True)
    assert max(i["off_rel"] for i in infos) <= 1e-14
    for k in np.random.default_rng(0).choice(len(sizes), 24, replace=False):
        n = int(sizes[k])
        A = packed[offs[k]:offs[k + 1]].astype(np.float64).reshape((n, n), order="F")
        check_against_oracle(A, Ws[k], Qs[k])
