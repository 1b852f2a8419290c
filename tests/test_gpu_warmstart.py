"""GPU parity of the learned warm start's kernels against the FP64 oracle
(oracle/mlp_oracle.py, oracle.cayley), and an end-to-end check that the
trained network lowers the sweep count of the batched solver.

Network bars, element by element: the oracle is the plain FP64 definition
(forward, and backward by the chain rule) evaluated on the weights the kernels
use (the BF16 copy of the master weights).  The kernels differ from it by the
BF16 rounding of their inputs and activations (unit roundoff u_b = 2^-8),
FP32 accumulation over K terms (K u_32 per product sum, u_32 = 2^-24) and the
FP32 GELU.  A running error bound carries these through the layers, entry by
entry (|H~ - H| <= E_H, then |Z~ - Z| <= E_H |W| + K u_32 (|H~| |W| + |b|),
GELU Lipschitz 1.129, GELU' Lipschitz 0.798, ...), and every output and
gradient entry must lie within twice its bound.  The oracle's `round_acts`
mode (the same quantisation points as the kernels) is printed as a diagnostic
only.  Adam: FP32 against FP64 (relative 1e-5), the BF16 copy bit-exact.
Cayley: 1e-13 against the long-double oracle.
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


UB, U32 = 2.0 ** -8, 2.0 ** -24   # unit roundoff of BF16 and FP32
LIP1, LIP2 = 1.129, 0.798         # max |gelu'|, max |gelu''| (tanh form)


def _gelu_eval_err(z):
    """Bound on |gelu32(z) - gelu(z)| for the FP32 evaluation
    0.5 z (1 + tanh(c (z + 0.044715 z^3))): argument error ~6 u_32 |a|, tanhf
    within 4 u_32, then 3 roundings of the products."""
    a = np.abs(M.C_GELU * (z + 0.044715 * z ** 3))
    return 0.5 * np.abs(z) * (6 * U32 * a + 4 * U32) + 3 * U32 * (np.abs(z) + 1.0)


def _gelu_grad_eval_err(z):
    a = np.abs(M.C_GELU * (z + 0.044715 * z ** 3))
    return 8 * U32 * (1.0 + np.abs(z) * (1.0 + a) * (1.0 + 3 * 0.044715 * z * z))


def forward_bounds(theta, Ws, bs):
    """Exact forward (FP64, no rounding) and entrywise bounds on the kernels'
    deviation from it: returns (Y, cache, EY, EH, EZ) with EH[l] bounding the
    kernels' layer-l input and EZ[l] its hidden pre-activation."""
    X = theta.astype(np.float64)
    Y, cache = M.forward(X, Ws, bs)
    EH = [np.abs(M.bf16(theta) - X)]          # the input is rounded to BF16
    EZ = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        K = W.shape[0] if l > 0 else 16       # the first layer's input is padded to 16 features
        H = cache["H"][l]
        Ez = EH[l] @ np.abs(W) + (K + 1) * U32 * ((np.abs(H) + EH[l]) @ np.abs(W) + np.abs(b))
        if l < len(Ws) - 1:
            Z = cache["Z"][l]
            e = LIP1 * Ez + _gelu_eval_err(np.abs(Z) + Ez)
            EH.append(e + UB * (np.abs(cache["H"][l + 1]) + e))
            EZ.append(Ez)
        else:
            EY = Ez
    return Y, cache, EY, EH, EZ


def backward_bounds(dY, Ws, cache, EH, EZ):
    """Exact gradients (chain rule in FP64 on the exact forward) and entrywise
    bounds on the kernels' deviation: dY rounded to BF16, FP32 accumulation,
    dZ = bf16((dZ W^T) gelu'(bf16(Z)))."""
    dWx, dbx = M.backward(dY, Ws, cache)
    L = len(Ws)
    B = dY.shape[0]
    D = dY.astype(np.float64)                 # exact dL/dZ of the current layer
    ED = np.abs(M.bf16(dY) - D)
    EW, Eb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        H = cache["H"][l]
        Ah, Ad = np.abs(H) + EH[l], np.abs(D) + ED
        EW[l] = EH[l].T @ np.abs(D) + Ah.T @ ED + B * U32 * (Ah.T @ Ad)
        Eb[l] = ED.sum(axis=0) + B * U32 * Ad.sum(axis=0)
        if l > 0:
            W = Ws[l]
            dH = D @ W.T
            EdH = ED @ np.abs(W).T + W.shape[1] * U32 * (Ad @ np.abs(W).T)
            Z = cache["Z"][l - 1]
            EZs = EZ[l - 1] + UB * (np.abs(Z) + EZ[l - 1])      # the saved Z is rounded to BF16
            Eg = LIP2 * EZs + _gelu_grad_eval_err(np.abs(Z) + EZs)
            g = M.gelu_grad(Z)
            Dn = dH * g
            e = EdH * np.abs(g) + (np.abs(dH) + EdH) * Eg
            ED = e + (UB + U32) * (np.abs(Dn) + e)
            D = Dn
    return dWx, dbx, EW, Eb


# BF16 activation slots of jws_mlp_forward / jws_mlp_backward (element offsets
# in units of the batch size B, row-major B x features; include/jacobi.h)
ACT = {"X0": (0, 16), "Z1": (16, 256), "H1": (272, 256), "Z2": (528, 256), "H2": (784, 256),
       "DZ2": (1040, 256), "DZ1": (1296, 256), "DY": (1552, 2016)}


def acts_of(net, B):
    """The kernels' saved BF16 tensors of the last forward / backward, as float64."""
    raw = net.acts(B).cpu().numpy().view(np.uint16)
    out = {}
    with np.errstate(invalid="ignore"):  # slots not written yet may hold NaN patterns
        for k, (o, w) in ACT.items():
            bits = raw[o * B:o * B + B * w].astype(np.uint32) << 16
            out[k] = bits.view(np.float32).astype(np.float64).reshape(B, w)
    return out


def _within(got, ref, bound, what):
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    ratio = float(np.max(err / (2.0 * bound + 1e-300)))
    assert np.all(err <= 2.0 * bound + 1e-300), (what, ratio)
    return ratio


@pytest.mark.parametrize("B", [37, 256])
def test_forward_matches_oracle(ws, B):
    import torch
    net, p = net_with_random_biases(ws, 1)
    theta = np.random.default_rng(2).normal(0, 0.1, (B, 8)).astype(np.float32)
    Y = net.forward(torch.from_numpy(theta).cuda()).cpu().numpy()
    Ws, bs = params_from_master(p)
    Yx, _, EY, _, _ = forward_bounds(theta, Ws, bs)
    r = _within(Y, Yx, EY, "Y")
    Yo, _ = M.forward(theta.astype(np.float64), Ws, bs, round_acts=True)
    print(f"forward B={B}: largest |dY| / (2 bound) {r:.3f}; relative error vs the exact definition "
          f"{rel(Y, Yx):.2e}, vs the kernels' quantisation points (diagnostic) {rel(Y, Yo):.2e}")
    # each layer against its definition on the kernels' own stored inputs:
    # Z = H W + b (FP32 accumulation: K u_32 (|H||W| + |b|)), stored in BF16
    # (u_b |Z|); H' = gelu(Z) in FP32, stored in BF16; Y = H2 W3 + b3 in FP32
    a = acts_of(net, B)
    np.testing.assert_array_equal(a["X0"][:, :8], M.bf16(theta))
    assert np.all(a["X0"][:, 8:] == 0.0)
    Hin = a["X0"][:, :8]
    worst = 0.0
    for l, (zk, hk) in enumerate((("Z1", "H1"), ("Z2", "H2"))):
        W, b = Ws[l], bs[l]
        K = 16 if l == 0 else W.shape[0]
        Z = Hin @ W + b
        ez = (K + 1) * U32 * (np.abs(Hin) @ np.abs(W) + np.abs(b))
        worst = max(worst, _within(a[zk], Z, 0.5 * (UB * (np.abs(Z) + ez) + ez), zk))
        Hn = M.gelu(Z)
        eh = LIP1 * ez + _gelu_eval_err(np.abs(Z) + ez)
        worst = max(worst, _within(a[hk], Hn, 0.5 * (UB * (np.abs(Hn) + eh) + eh), hk))
        Hin = a[hk]
    Yl = Hin @ Ws[2] + bs[2]
    worst = max(worst, _within(Y, Yl, 0.5 * (257 * U32 * (np.abs(Hin) @ np.abs(Ws[2]) + np.abs(bs[2]))), "Y layer"))
    print(f"  per layer, largest |err| / bound {2 * worst:.3f}")


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
    Yk = Y.cpu().numpy().astype(np.float64)
    # the loss of the kernels' own outputs (FP32 differences, FP64 sum)
    assert abs(float(loss.item()) - M.mse(Yk, T)) <= 1e-6 * M.mse(Yk, T)
    dYn = dY.cpu().numpy()
    Yx, cx, _, EH, EZ = forward_bounds(theta, Ws, bs)
    dWx, dbx, EW, Eb = backward_bounds(dYn, Ws, cx, EH, EZ)
    gW1 = g[OFF_W1:OFF_W2].reshape(16, 256)
    assert np.all(gW1[8:] == 0.0)          # padded input features get no gradient
    got = [gW1[:8], g[OFF_W2:OFF_W3].reshape(256, 256), g[OFF_W3:OFF_B1].reshape(256, 2016)]
    gb = g[OFF_B1:]
    gotb = [gb[:256], gb[256:512], gb[512:]]
    _, co = M.forward(theta.astype(np.float64), Ws, bs, round_acts=True)
    dWo, dbo = M.backward(dYn.astype(np.float64), Ws, co, round_acts=True)
    for l in range(3):
        rw = _within(got[l], dWx[l], EW[l], f"dW{l + 1}")
        rb = _within(gotb[l], dbx[l], Eb[l], f"db{l + 1}")
        print(f"backward B={B} layer {l + 1}: largest |err| / (2 bound) dW {rw:.3f} db {rb:.3f}; relative error "
              f"vs exact dW {rel(got[l], dWx[l]):.2e}, vs the kernels' quantisation points (diagnostic) "
              f"{rel(got[l], dWo[l]):.2e}")
    # each step against its definition on the kernels' own stored operands:
    # dW = H^T dZ and db = colsum dZ (FP32 accumulation over the batch),
    # dZ_prev = (dZ W^T) * gelu'(Z) (FP32, stored in BF16)
    a = acts_of(net, B)
    np.testing.assert_array_equal(a["DY"], M.bf16(dYn))
    Hs, Ds = [a["X0"][:, :8], a["H1"], a["H2"]], [a["DZ1"], a["DZ2"], a["DY"]]
    worst = 0.0
    for l in range(3):
        H, D = Hs[l], Ds[l]
        worst = max(worst, _within(got[l], H.T @ D, 0.5 * (B + 1) * U32 * (np.abs(H).T @ np.abs(D)), f"dW{l + 1} step"))
        worst = max(worst, _within(gotb[l], D.sum(0), 0.5 * (B + 1) * U32 * np.abs(D).sum(0), f"db{l + 1} step"))
        if l > 0:
            W, Zs = Ws[l], a["Z1" if l == 1 else "Z2"]
            dH = D @ W.T
            ed = (W.shape[1] + 1) * U32 * (np.abs(D) @ np.abs(W).T)
            g = M.gelu_grad(Zs)
            ref = dH * g
            e = ed * np.abs(g) + (np.abs(dH) + ed) * _gelu_grad_eval_err(np.abs(Zs))
            worst = max(worst, _within(Ds[l - 1], ref, 0.5 * ((UB + U32) * (np.abs(ref) + e) + e), f"dZ{l} step"))
    print(f"  per step, largest |err| / bound {2 * worst:.3f}")


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


def test_family_matrices_match_definition(ws):
    import torch
    from paper_2608_28952_amd import inputs
    fam = ws.Family(5)
    th = inputs.warmstart_thetas(33, 7)
    A = fam.matrices(th).cpu().numpy()
    ref = inputs.warmstart_matrices(fam.A0, fam.B, th)
    assert np.max(np.abs(A - ref)) <= 1e-15 * 16 * np.max(np.abs(ref))


def test_canonical_targets_match_oracle(ws):
    """The kernel's canonical generators against the oracle's plain definition
    (greedy overlap matching by loops, signs, np.linalg.det, the inverse
    Cayley map by np.linalg.solve), sample by sample: the kept flag exactly,
    the FP32 coordinates within one FP32 rounding of the FP64 values (plus
    1e-12).  Solutions of family members (eigh of the same inputs), some with
    columns permuted and negated, and a few unrelated orthogonal matrices
    (targets far from Qref, typically dropped)."""
    import torch
    from paper_2608_28952_amd import inputs
    fam = ws.Family(5)
    Qref = fam.Qref.cpu().numpy()
    th = inputs.warmstart_thetas(40, 11)
    A = inputs.warmstart_matrices(fam.A0, fam.B, th)
    rng = np.random.default_rng(12)
    Qs = [np.linalg.eigh(a)[1] for a in A]
    for k in range(0, 40, 5):
        Qs[k] = Qs[k][:, rng.permutation(64)] * rng.choice([-1.0, 1.0], 64)
    Qs += [inputs.haar(64, rng) for _ in range(6)]
    Q = torch.from_numpy(np.ascontiguousarray(np.stack(Qs))).cuda()
    coords, keep = ws.canonical_targets(fam, Q)
    coords, keep = coords.cpu().numpy(), keep.cpu().numpy()
    for k, q in enumerate(Qs):
        S, _ = M.canonical_generator(Qref, q)
        ok = bool(np.all(np.isfinite(S)) and np.max(np.abs(S)) <= 10.0)
        assert bool(keep[k]) == ok, k
        if ok:
            c = M.coords_from_skew(S)
            assert np.all(np.abs(coords[k] - c) <= 2.0 ** -23 * np.abs(c) + 1e-12), k
        else:
            assert np.all(coords[k] == 0.0)
    print(f"kept {int(keep.sum())} of {len(Qs)}")


def test_column_stats_and_standardize_match_definition(ws):
    import torch
    rng = np.random.default_rng(13)
    rows = 2500
    X = rng.standard_normal((rows, 8)).astype(np.float32)
    C = (rng.standard_normal((rows, 2016)) * 0.3 + 0.1).astype(np.float32)
    keep = (rng.random(rows) < 0.8).astype(np.int32)
    Xo, To, (mean, std) = ws.standardized(torch.from_numpy(X).cuda(), torch.from_numpy(C).cuda(),
                                          torch.from_numpy(keep).cuda())
    k = keep.astype(bool)
    mu = C[k].astype(np.float64).mean(0)
    sd = C[k].astype(np.float64).std(0) + 1e-6
    assert np.max(np.abs(mean.cpu().numpy() - mu)) <= 1e-6 * np.max(np.abs(mu))
    assert np.max(np.abs(std.cpu().numpy() - sd) / sd) <= 1e-6
    np.testing.assert_array_equal(Xo.cpu().numpy(), X[k])
    T = (C[k] - mean.cpu().numpy()) / std.cpu().numpy()
    assert np.max(np.abs(To.cpu().numpy() - T)) <= 1e-6 * np.max(np.abs(T))


def test_training_and_warm_start_gain(ws):
    """Reduced-size pipeline (16384 training samples, 10 epochs): the loss
    falls, and on held-out parameters the network's starts take fewer sweeps
    than the cold start and than the two starts that use no network (Qref,
    and Qref cay(S_mean)), with results that match the oracle."""
    import torch
    fam = ws.Family(5)
    th, coords, keep = ws.generate(fam, 16384, 50)
    vth, vco, vkeep = ws.generate(fam, 1024, 51)
    X, T, stats = ws.standardized(th, coords, keep)
    VX, VT, _ = ws.standardized(vth, vco, vkeep, stats=stats)
    net = ws.Net(seed=0)
    net.mean, net.std = stats
    v0 = float(net.mse(net.forward(VX), VT).item())
    tr = ws.train(net, X, T, VX, VT, epochs=10, log=print)
    print(f"kept {X.shape[0]} of 16384; val loss {v0:.3e} -> {tr['best_val']:.3e} in {tr['seconds']:.1f}s")
    assert tr["best_val"] < 0.9 * v0
    test_theta = np.random.default_rng(52).normal(0, 0.1, (512, 8))
    ev = ws.evaluate(net, fam, test_theta, reps=1)
    print({k: (v["sweeps_mean"], v["fallback_rate"]) if isinstance(v, dict) else v for k, v in ev.items()})
    assert ev["status_ok"]
    assert ev["network"]["sweeps_mean"] < ev["cold"]["sweeps_mean"]
    assert ev["network"]["sweeps_mean"] < ev["qref"]["sweeps_mean"]
    assert ev["network"]["sweeps_mean"] < ev["mean_generator"]["sweeps_mean"]
    # warm-started results against the oracle on a few matrices
    A = fam.matrices(test_theta[:4])
    W, Q, infos = ws.solve(A, Q0=ws.propose(net, fam, torch.from_numpy(test_theta[:4].astype(np.float32)).cuda()))
    for k in range(4):
        Ak = A[k].cpu().numpy()
        ora = O.eig(Ak)
        assert np.max(np.abs(W[k].cpu().numpy() - ora.W)) <= 1e-12 * np.max(np.abs(ora.W))
        res, orth, _, _ = O.check_eig(Ak, W[k].cpu().numpy(), np.asfortranarray(Q[k].cpu().numpy()))
        assert res <= 1e-12 and orth <= 1e-12
