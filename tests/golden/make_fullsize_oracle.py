"""Write the oracle's results on the full-size workloads as text fixtures.

Calls only the CPU oracle (oracle/) and the seeded input generators; nothing
here touches the GPU library.  The GPU tests compare the library's results at
these sizes with the files written here.

    python tests/golden/make_fullsize_oracle.py [--threads T] [--only NAME ...]

Fixtures (one value per line, 17 significant digits, '#' header lines):
  eig_graded_n4096_seed2.txt   eigenvalues, ascending, of the graded n = 4096
                               matrix (lambda_i = +-10^(-8 i / n), Haar Q,
                               seed 2): scalar cyclic Jacobi (Alg. 1 with
                               b = 1), round-robin rounds, to
                               Xi(A) <= 1e-14 ||A||_F (eq. Omega_A, §2.1)
  eig_uniform_n2048_seed7.txt  the same for n = 2048, lambda ~ U[-1, 1], seed 7
  svd_16384x2048_seed3.txt     singular values, descending, of G = U diag(s) V^T
                               (16384 x 2048, s = 10^U(-6, 0), seed 3): one-sided
                               Hestenes Jacobi (Alg. 6 with b = 1), round-robin
                               rounds, until a sweep rotates no pair
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_28952_amd import inputs  # noqa: E402


def _write(name, header, values):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        for v in values:
            f.write(f"{float(v):.17g}\n")
    print(f"wrote {path}", flush=True)


def eig_fixture(name, A, desc, threads):
    t0 = time.time()
    r = O.eig(A, tol=1e-14, max_sweeps=50, order=1, want_vectors=False, nthreads=threads)
    dt = time.time() - t0
    assert r.status == 0, r.status
    _write(name, [desc,
                  "oracle: scalar cyclic Jacobi (Alg. 1 with b = 1), round-robin rounds, FP64, "
                  "stop at Xi(A) <= 1e-14 ||A||_F (eq. Omega_A, §2.1)",
                  f"sweeps {r.sweeps}, rotations {r.rotations}, {threads} threads, {dt:.0f} s",
                  "written by tests/golden/make_fullsize_oracle.py; eigenvalues ascending"], r.W)


def svd_fixture(name, G, desc, threads):
    t0 = time.time()
    r = O.svd(G, order=1, nthreads=threads)
    dt = time.time() - t0
    assert r.status == 0, r.status
    _write(name, [desc,
                  "oracle: one-sided Hestenes Jacobi (Alg. 6 with b = 1), round-robin rounds, FP64, "
                  "rotate when |g_p^T g_q| > sqrt(m) eps |g_p| |g_q|, stop when a sweep rotates none",
                  f"sweeps {r.sweeps}, rotations {r.rotations}, {threads} threads, {dt:.0f} s",
                  "written by tests/golden/make_fullsize_oracle.py; singular values descending"], r.S)


FIXTURES = {
    "eig_uniform_n2048_seed7": lambda t: eig_fixture(
        "eig_uniform_n2048_seed7.txt", inputs.eig_uniform(2048, 7)[0],
        "A = Q diag(lambda) Q^T, n = 2048, Q Haar, lambda ~ U[-1, 1], seed 7 (inputs.eig_uniform)", t),
    "svd_16384x2048_seed3": lambda t: svd_fixture(
        "svd_16384x2048_seed3.txt", inputs.svd_case(16384, 2048, 3)[0],
        "G = U diag(s) V^T, 16384 x 2048, U, V Haar, s = 10^U(-6, 0), seed 3 (inputs.svd_case)", t),
    "eig_graded_n4096_seed2": lambda t: eig_fixture(
        "eig_graded_n4096_seed2.txt", inputs.eig_graded(4096, 2)[0],
        "A = Q diag(lambda) Q^T, n = 4096, Q Haar, lambda_i = +-10^(-8 i / n), seed 2 (inputs.eig_graded)", t),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    for name, fn in FIXTURES.items():
        if args.only and name not in args.only:
            continue
        print(f"{name} ...", flush=True)
        fn(args.threads)


if __name__ == "__main__":
    main()
