"""GPU parity of the learned warm start's kernels against the FP64 oracle
(oracle/mlp_oracle.py, oracle.cayley), and an end-to-end check that the
trained network lowers the sweep count of the batched solver.

Bars: the network kernels see BF16 operands; the oracle is evaluated on the
same BF16-rounded weights and activations in FP64, so the remaining
differences are FP32 accumulation order and FP32 GELU (relative Frobenius
error <= 2e-3 per tensor, against 2^-8 = 3.9e-3 for a single BF16 rounding).
Against the exact FP64 gradient (no rounding) the error is reported and held
below 5e-2.  Adam: FP32 against FP64 (relative 1e-5), the BF16 copy
bit-exact.  Cayley: 1e-13 against the long-double oracle.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import oracle as O

pytestmark = pytest.mark.gpu

NPARAM = 588256
OFF_W1, OFF_W2, OFF_W3, OFF_B1 = 0, 4096, 69632, 585728


@pytest.fixture(scope="module")
def ws():
    import torch
    from paper_2608_28952_amd import jacobi, warmstart
    assert torch.cuda.is_available()
    jacobi.lib()
    return warmstart


def params_from_master(p, bf16=True):
    r = M.bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1 = r(p[OFF_W1:OFF_W2]).reshape(16, 256)[:8]
    W2 = r(p[OFF_W2:OFF_W3]).reshape(256, 256)
    W3 = r(p[OFF_W3:OFF_B1]).reshape(256, 2016)
    b = p[OFF_B1:].astype(np.float64)
    return [W1, W2, W3], [b[:256], b[256:512], b[512:]]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def net_with_random_biases(ws, seed):
    import torch
    net = ws.Net(seed=seed)
    rng = np.random.default_rng(seed + 100)
    p = net.master.cpu().numpy()
    p[OFF_B1:] = rng.standard_normal(NPARAM - OFF_B1).astype(np.float32) * 0.1
    net.master.copy_(torch.from_numpy(p))
    from paper_2608_28952_amd import jacobi as jx
    jx.lib().jws_to_bf16(NPARAM, net.master.data_ptr(), net.bf16.data_ptr(), None)
    return net, p


@pytest.mark.parametrize("B", [37, 256])
def test_forward_matches_oracle(ws, B):
    import torch
    net, p = net_with_random_biases(ws, 1)
    theta = np.random.default_rng(2).normal(0, 0.1, (B, 8)).astype(np.float32)
    Y = net.forward(torch.from_numpy(theta).cuda()).cpu().numpy()
    Ws, bs = params_from_master(p)
    Yo, _ = M.forward(theta.astype(np.float64), Ws, bs, round_acts=True)
    e = rel(Y, Yo)
    print(f"forward B={B}: relative error {e:.2e}")
    assert e <= 2e-3


@pytest.mark.parametrize("B", [37, 512])
def test_backward_matches_oracle(ws, B):
    import torch
    net, p = net_with_random_biases(ws, 3)
    rng = np.random.default_rng(4)
    theta = rng.normal(0, 0.1, (B, 8)).astype(np.float32)
    T = rng.standard_normal((B, 2016)).astype(np.float32)
    th = torch.from_numpy(theta).cuda()
    Y = net.forward(th)
    dY = torch.empty_like(Y)
    loss = net.mse(Y, torch.from_numpy(T).cuda(), dY=dY)
    net.backward(th, dY)
    g = net.grad.cpu().numpy()
    Ws, bs = params_from_master(p)
    Yo, cache = M.forward(theta.astype(np.float64), Ws, bs, round_acts=True)
    assert abs(float(loss.item()) - M.mse(Yo, T)) <= 1e-3 * M.mse(Yo, T)
    dWo, dbo = M.backward(dY.cpu().numpy().astype(np.float64), Ws, cache, round_acts=True)
    gW1 = g[OFF_W1:OFF_W2].reshape(16, 256)
    assert np.all(gW1[8:] == 0.0)          # padded input features get no gradient
    got = [gW1[:8], g[OFF_W2:OFF_W3].reshape(256, 256), g[OFF_W3:OFF_B1].reshape(256, 2016)]
    gb = g[OFF_B1:]
    gotb = [gb[:256], gb[256:512], gb[512:]]
    for l in range(3):
        ew, eb = rel(got[l], dWo[l]), rel(gotb[l], dbo[l])
        print(f"backward B={B} layer {l + 1}: dW {ew:.2e} db {eb:.2e}")
        assert ew <= 2e-3 and eb <= 2e-3
    # against the exact FP64 gradient of the same parameters (no rounding)
    Wx, bx = params_from_master(p, bf16=False)
    Yx, cx = M.forward(theta.astype(np.float64), Wx, bx)
    dWx, dbx = M.backward(M.mse_grad(Yx, T.astype(np.float64)), Wx, cx)
    ex = max(rel(got[l], dWx[l]) for l in range(3))
    print(f"gradient-check error vs exact FP64 (B={B}): {ex:.2e}")
    assert ex <= 5e-2


def test_adam_matches_oracle(ws):
    import torch
    from paper_2608_28952_amd import jacobi as jx
    rng = np.random.default_rng(7)
    n = 100003
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 0.1).astype(np.float32)
    v = (rng.random(n) * 0.01).astype(np.float32)
    dp, dg, dm, dv = (torch.from_numpy(x.copy()).cuda() for x in (p, g, m, v))
    db = torch.empty(n, dtype=torch.int16, device="cuda")
    rc = jx.lib().jws_adam_step(n, dp.data_ptr(), db.data_ptr(), dg.data_ptr(), dm.data_ptr(), dv.data_ptr(),
                                1e-3, 0.9, 0.999, 1e-8, 3, None)
    assert rc == 0
    # the kernel's hyperparameters are FP32: the reference uses the same values
    f = lambda x: float(np.float32(x))
    po, mo, vo = M.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                             f(1e-3), f(0.9), f(0.999), f(1e-8), 3)
    gp, gm, gv = dp.cpu().numpy(), dm.cpu().numpy(), dv.cpu().numpy()
    assert rel(gm, mo) <= 1e-6 and rel(gv, vo) <= 1e-6
    assert np.max(np.abs(gp - po) / np.maximum(np.abs(po), 1e-3)) <= 1e-5
    assert np.array_equal(db.cpu().numpy().view(np.uint16), M.bf16_bits(gp))


def test_mse_matches_definition(ws):
    import torch
    net = ws.Net(seed=0)
    rng = np.random.default_rng(8)
    Y = rng.standard_normal((33, 2016)).astype(np.float32)
    T = rng.standard_normal((33, 2016)).astype(np.float32)
    dY = torch.empty(33, 2016, dtype=torch.float32, device="cuda")
    loss = net.mse(torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda(), dY=dY)
    d = Y.astype(np.float64) - T
    # Y - T is formed in FP32 (relative error 2^-24 per entry), squares summed in FP64
    assert abs(float(loss.item()) - np.mean(d * d)) <= 1e-6 * np.mean(d * d)
    assert np.max(np.abs(dY.cpu().numpy() - 2 * d / d.size)) <= 1e-6 * np.max(np.abs(2 * d / d.size))


def test_skew_and_cayley_match_oracle(ws):
    import torch
    from paper_2608_28952_amd import jacobi as jx
    rng = np.random.default_rng(9)
    B, n = 5, 64
    c = rng.standard_normal((B, 2016)).astype(np.float32)
    mean = (rng.standard_normal(2016) * 0.01).astype(np.float32)
    std = (rng.random(2016) * 0.05).astype(np.float32)
    S = torch.empty(B, n, n, dtype=torch.float64, device="cuda")
    tc, tm, ts = (torch.from_numpy(x).cuda() for x in (c, mean, std))
    assert jx.lib().jws_skew_from_coords(B, n, tc.data_ptr(), tm.data_ptr(), ts.data_ptr(), S.data_ptr(), None) == 0
    Scm = S.cpu().numpy()   # [k] holds the column-major matrix: Scm[k][j][i] = S_k(i, j)
    Qref = np.linalg.qr(rng.standard_normal((n, n)))[0]
    Q0 = torch.empty(B, n, n, dtype=torch.float64, device="cuda")
    qref = torch.from_numpy(np.ascontiguousarray(Qref.T)).cuda()   # column-major storage
    assert jx.lib().jws_cayley_batched(B, n, S.data_ptr(), qref.data_ptr(), Q0.data_ptr(), None) == 0
    Q0 = Q0.cpu().numpy()
    for k in range(B):
        Sk = Scm[k].T
        coords = c[k].astype(np.float64) * std + mean
        assert np.max(np.abs(Sk - M.skew_from_coords(coords))) <= 1e-6 * np.max(np.abs(coords))
        assert np.array_equal(Sk, -Sk.T)
        ref = Qref @ O.cayley(Sk)
        got = Q0[k].T
        assert np.max(np.abs(got - ref)) <= 1e-13, np.max(np.abs(got - ref))
        assert np.linalg.norm(got.T @ got - np.eye(n)) <= 1e-13
    # 2 x 2 closed form: cay([[0, s], [-s, 0]]) = [[1 - s^2, 2s], [-2s, 1 - s^2]] / (1 + s^2)
    s = 0.3
    S2 = torch.tensor([[0.0, -s], [s, 0.0]], dtype=torch.float64, device="cuda")  # column-major [[0, s], [-s, 0]]
    I2 = torch.eye(2, dtype=torch.float64, device="cuda")
    out = torch.empty(2, 2, dtype=torch.float64, device="cuda")
    assert jx.lib().jws_cayley_batched(1, 2, S2.data_ptr(), I2.data_ptr(), out.data_ptr(), None) == 0
    ref2 = np.array([[1 - s * s, 2 * s], [-2 * s, 1 - s * s]]) / (1 + s * s)
    assert np.max(np.abs(out.cpu().numpy().T - ref2)) <= 1e-15


def test_training_and_warm_start_gain(ws):
    """Reduced-size pipeline (8192 training samples, 8 epochs): the loss falls,
    and warm starts on held-out parameters take fewer sweeps than cold starts,
    with results that match the oracle."""
    import torch
    fam = ws.Family(5)
    th, coords, keep = ws.generate(fam, 8192, 50)
    vth, vco, vkeep = ws.generate(fam, 1024, 51)
    mean, std = coords[keep].mean(0), coords[keep].std(0) + 1e-6
    net = ws.Net(seed=0)
    net.mean, net.std = torch.from_numpy(mean).cuda(), torch.from_numpy(std).cuda()
    X, T = torch.from_numpy(th[keep]).cuda(), torch.from_numpy((coords[keep] - mean) / std).cuda()
    VX, VT = torch.from_numpy(vth[vkeep]).cuda(), torch.from_numpy((vco[vkeep] - mean) / std).cuda()
    v0 = float(net.mse(net.forward(VX), VT).item())
    tr = ws.train(net, X, T, VX, VT, epochs=8, log=print)
    print(f"dropped {1 - keep.mean():.3f}; val loss {v0:.3e} -> {tr['best_val']:.3e} in {tr['seconds']:.1f}s")
    assert tr["best_val"] < 0.9 * v0
    test_theta = np.random.default_rng(52).normal(0, 0.1, (512, 8))
    ev = ws.evaluate(net, fam, test_theta, reps=1)
    print(ev)
    assert ev["status_ok"]
    assert ev["warm_sweeps_mean"] < ev["cold_sweeps_mean"]
    # warm-started results against the oracle on a few matrices
    A = fam.matrices(test_theta[:4])
    W, Q, infos = ws.solve(A, Q0=ws.propose(net, fam, torch.from_numpy(test_theta[:4].astype(np.float32)).cuda()))
    for k in range(4):
        Ak = A[k].cpu().numpy()
        ora = O.eig(Ak)
        assert np.max(np.abs(W[k].cpu().numpy() - ora.W)) <= 1e-12 * np.max(np.abs(ora.W))
        res, orth, _, _ = O.check_eig(Ak, W[k].cpu().numpy(), np.asfortranarray(Q[k].cpu().numpy()))
        assert res <= 1e-12 and orth <= 1e-12
