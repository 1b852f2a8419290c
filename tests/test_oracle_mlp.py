"""Pins of the FP64 network reference (oracle/mlp_oracle.py): central finite
differences for every parameter tensor, the closed-form gradient of a linear
layer, GELU against its definition and limits, Adam's first step, BF16
rounding on known bit patterns, and the canonical generator round trip."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import oracle as O


def small_net(seed, sizes=(3, 5, 4, 6)):
    rng = np.random.default_rng(seed)
    Ws, bs = M.init_params(rng, sizes)
    bs = [rng.standard_normal(b.shape) * 0.1 for b in bs]
    X = rng.standard_normal((7, sizes[0]))
    T = rng.standard_normal((7, sizes[-1]))
    return Ws, bs, X, T


def loss(Ws, bs, X, T):
    Y, _ = M.forward(X, Ws, bs)
    return M.mse(Y, T)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    Ws, bs, X, T = small_net(seed)
    Y, cache = M.forward(X, Ws, bs)
    dWs, dbs = M.backward(M.mse_grad(Y, T), Ws, cache)
    h = 1e-6
    for tensors, grads in ((Ws, dWs), (bs, dbs)):
        for P, G in zip(tensors, grads):
            num = np.zeros_like(P)
            for idx in np.ndindex(P.shape):
                old = P[idx]
                P[idx] = old + h
                lp = loss(Ws, bs, X, T)
                P[idx] = old - h
                lm = loss(Ws, bs, X, T)
                P[idx] = old
                num[idx] = (lp - lm) / (2 * h)
            assert np.max(np.abs(num - G)) <= 1e-8 * max(1.0, np.max(np.abs(G)))


def test_linear_layer_closed_form():
    # one linear layer, L = mean((XW + b - T)^2): dW = 2 X^T (Y - T) / (B N)
    rng = np.random.default_rng(3)
    X, W, b, T = rng.standard_normal((6, 4)), rng.standard_normal((4, 3)), rng.standard_normal(3), rng.standard_normal((6, 3))
    Y, cache = M.forward(X, [W], [b])
    dWs, dbs = M.backward(M.mse_grad(Y, T), [W], cache)
    assert np.allclose(dWs[0], 2 * X.T @ (X @ W + b - T) / 18, rtol=0, atol=1e-14)
    assert np.allclose(dbs[0], 2 * (X @ W + b - T).sum(0) / 18, rtol=0, atol=1e-14)


def test_gelu_definition_and_limits():
    z = np.linspace(-6, 6, 101)
    ref = 0.5 * z * (1 + np.tanh(np.sqrt(2 / np.pi) * (z + 0.044715 * z ** 3)))
    assert np.array_equal(M.gelu(z), ref)
    assert M.gelu(0.0) == 0.0 and abs(M.gelu(20.0) - 20.0) < 1e-12 and abs(M.gelu(-20.0)) < 1e-12
    h = 1e-6
    assert np.max(np.abs((M.gelu(z + h) - M.gelu(z - h)) / (2 * h) - M.gelu_grad(z))) < 1e-8
    assert abs(M.gelu_grad(0.0) - 0.5) < 1e-15


def test_adam_first_step_moves_by_lr():
    # after one step with bias correction, |dp| = lr * |g| / (|g| + eps) per entry
    g = np.array([1e-3, -2.0, 5.0])
    p, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # zero gradient leaves the parameter unchanged
    p2, _, _ = M.adam_step(np.ones(2), np.zeros(2), np.zeros(2), np.zeros(2), 1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.array_equal(p2, np.ones(2))


def test_bf16_rounding_known_patterns():
    # BF16 keeps 8 significant bits: the spacing above 1.0 is 2^-7
    x = np.array([1.0, -2.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 1.0 + 2 ** -8 + 2 ** -20, 3.0e38, 0.0],
                 dtype=np.float32)
    bits = M.bf16_bits(x)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6)
    assert list(bits[:4]) == [0x3F80, 0xC000, 0x3F80, 0x3F82]
    assert bits[4] == 0x3F80 and bits[5] == 0x3F81   # below / above the halfway point
    assert bits[7] == 0 and M.bf16(np.float32(np.inf)) == np.inf
    assert np.isnan(M.bf16(np.float32(np.nan)))
    # rounding error bound u = 2^-8 relative
    r = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    assert np.max(np.abs(M.bf16(r) - r) / np.abs(r)) <= 2.0 ** -8


def test_skew_coordinates_round_trip():
    rng = np.random.default_rng(4)
    c = rng.standard_normal(2016)
    S = M.skew_from_coords(c)
    assert np.array_equal(S, -S.T) and np.array_equal(M.coords_from_skew(S), c)
    assert S[0, 1] == c[0] and S[0, 63] == c[62] and S[1, 2] == c[63] and S[62, 63] == c[-1]


def test_greedy_match_on_permutation_and_brute_force():
    rng = np.random.default_rng(6)
    P = np.eye(5)[:, rng.permutation(5)] * rng.choice([-1.0, 1.0], 5)
    c = M.greedy_match(P + 0.01 * rng.standard_normal((5, 5)))
    assert np.all(np.abs(P[np.arange(5), c]) == 1.0)
    # on a diagonally dominant matrix the greedy choice is the identity
    D = np.eye(6) * 3 + rng.random((6, 6))
    assert M.greedy_match(D) == list(range(6))


def test_canonical_generator_inverts_cayley():
    # Q = Qref cay(S) with a small S: the canonical target gives S back, and
    # sign flips / column order of Q do not change it
    rng = np.random.default_rng(5)
    n = 64
    Qref = np.linalg.qr(rng.standard_normal((n, n)))[0]
    S = M.skew_from_coords(rng.standard_normal(2016) * 0.02)
    Q = Qref @ O.cayley(S)
    S1, W = M.canonical_generator(Qref, Q)
    assert np.max(np.abs(S1 - S)) < 1e-12
    flips = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    S2, _ = M.canonical_generator(Qref, Q * flips)
    assert np.max(np.abs(S2 - S)) < 1e-12
    S3, _ = M.canonical_generator(Qref, (Q * flips)[:, rng.permutation(n)])
    assert np.max(np.abs(S3 - S)) < 1e-12
    assert np.linalg.det(W) > 0 and np.all(np.diag(W) >= 0)
