"""Host-side logic of the warm start: the training targets the package builds
(vectorised overlap matching, sign and determinant fix, inverse Cayley)
agree with the oracle's plain definition."""
import numpy as np

from oracle import mlp_oracle as M
from paper_2608_28952_amd import inputs
from paper_2608_28952_amd import warmstart as W


def test_canonical_targets_match_oracle_definition():
    A0, B = inputs.warmstart_family(5, 64, 8)
    _, Qref = np.linalg.eigh(A0)
    th = inputs.warmstart_thetas(60, 50)
    As = inputs.warmstart_matrices(A0, B, th)
    Qs = np.array([np.linalg.eigh(A)[1] for A in As])
    coords, keep = W.canonical_targets(Qref, Qs, chunk=16)
    assert keep.mean() >= 0.9
    for k in range(len(As)):
        S, Wm = M.canonical_generator(Qref, Qs[k])
        assert keep[k] == (np.max(np.abs(S)) <= 10.0)
        if keep[k]:
            assert np.max(np.abs(coords[k] - M.coords_from_skew(S))) <= 1e-6 * max(1.0, np.max(np.abs(S)))


def test_greedy_columns_match_oracle():
    rng = np.random.default_rng(1)
    Wb = rng.standard_normal((7, 64, 64))
    c = W._greedy_columns(Wb)
    for k in range(7):
        assert list(c[k]) == M.greedy_match(Wb[k])
