"""Learned warm start for batched Jacobi on a parametrised matrix family.

An addition to the paper's method, which has no learned part: for the
family A(theta) = A0 + sum_k theta_k B_k (order 64, theta in R^8), a small
network proposes Q0 = Qref cay(S(theta)) and the batched Jacobi solver
finishes from Q0^T A Q0; a proposal that does not lower the off-norm falls
back to the cold start inside the solver.

Every numerical step runs in the library's kernels (through the C-ABI): the
family's matrices (jws_family_matrices), the batched FP64 solver that
generates the training solutions, their canonical targets
(jws_canonical_targets), the target statistics and standardisation
(jws_column_stats, jws_gather_standardize), the network's training
(jws_mlp_forward / jws_mlp_backward / jws_mse / jws_adam_step) and the
proposals (jws_skew_from_coords, jws_cayley_batched).  PyTorch holds device
memory; the host only draws the seeded parameters and keeps index lists.

    python -m paper_2608_28952_amd.warmstart [--train 262144] [--epochs 40]
"""
import argparse
import json
import time

import numpy as np

from . import inputs
from . import jacobi as jx

N = 64
NC = N * (N - 1) // 2  # 2016 generator coordinates
NIN, K1, HID = 8, 16, 256
OFF_W1, OFF_W2, OFF_W3 = 0, K1 * HID, K1 * HID + HID * HID
OFF_B1 = OFF_W3 + HID * NC
NPARAM = OFF_B1 + 2 * HID + NC


def _p(t):
    return None if t is None else t.data_ptr()


def _s():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _chk(rc, what):
    if rc != 0:
        raise jx.JacobiError(rc, f"{what}: {jx.last_error()}")


# ---------------------------------------------------------------------------
# Family, solutions and targets
# ---------------------------------------------------------------------------
class Family:
    """A0, B_1..B_8 (seeded symmetric N(0, 1/n)) and Qref = eigenvectors of A0
    (ascending eigenvalues), computed by the library's eigensolver."""

    def __init__(self, seed=5):
        import torch
        self.A0, self.B = inputs.warmstart_family(seed, N, NIN)
        A0 = torch.from_numpy(np.ascontiguousarray(self.A0)).cuda()
        _, Qref, _ = jx.jacobi_eig(A0)
        self.Qref = Qref.contiguous()                    # n x n (row-major view of the matrix)
        self.Qref_cm = Qref.t().contiguous()             # column-major storage for the kernels
        self.Bt = torch.from_numpy(np.ascontiguousarray(self.B)).cuda()   # 8 x n x n
        self.A0t = A0

    def matrices(self, theta):
        """theta: m x 8 (numpy or CUDA tensor) -> m x n x n FP64 CUDA tensor
        A0 + sum_k theta_k B_k (symmetric, so row- and column-major storage
        coincide), formed by jws_family_matrices."""
        import torch
        th = torch.as_tensor(theta, dtype=torch.float64, device="cuda").contiguous()
        m = th.shape[0]
        A = torch.empty(m, N, N, dtype=torch.float64, device="cuda")
        _chk(jx.lib().jws_family_matrices(m, N, NIN, _p(th), _p(self.A0t), _p(self.Bt), _p(A), _s()),
             "jws_family_matrices")
        return A


def solve(A, Q0=None, precision=None, max_sweeps=60):
    """Batched FP64 solve of m x n x n matrices; returns (W m x n, Q m x n x n
    with Q[k] the eigenvector matrix, per-matrix info as a numpy structured
    array)."""
    import torch
    m = A.shape[0]
    sizes = np.full(m, N, dtype=np.int32)
    offs = np.arange(m + 1, dtype=np.int64) * N * N
    o = jx.opts_default(precision=jx.PREC_FP64 if precision is None else precision, max_sweeps=max_sweeps)
    ws = torch.empty(jx.batched_workspace(sizes, True, o), dtype=torch.uint8, device="cuda")
    q0 = None if Q0 is None else Q0.transpose(1, 2).contiguous().reshape(-1)
    W, Q, infos = jx.jacobi_eig_batched(sizes, offs, A.reshape(-1), Q0=q0, opts=o, work=ws, info="array")
    return W.view(m, N), Q.view(m, N, N).transpose(1, 2), infos


def canonical_targets(fam, Q, maxabs=10.0):
    """Generator coordinates of solved matrices (m x n x n CUDA tensor, Q[k] the
    eigenvector matrix, eigenvalues ascending): jws_canonical_targets (overlap
    matching to Qref, signs, determinant, inverse Cayley).  Returns (coords
    m x 2016 FP32 CUDA, keep m int32 CUDA: finite and max |S_ij| <= maxabs)."""
    import torch
    m = Q.shape[0]
    Qcm = Q.transpose(1, 2).contiguous()   # column-major storage of each matrix
    coords = torch.empty(m, NC, dtype=torch.float32, device="cuda")
    keep = torch.empty(m, dtype=torch.int32, device="cuda")
    _chk(jx.lib().jws_canonical_targets(m, N, _p(Qcm), _p(fam.Qref_cm), _p(coords), _p(keep), maxabs, _s()),
         "jws_canonical_targets")
    return coords, keep


def standardized(theta, coords, keep, stats=None, eps=1e-6):
    """Kept rows of (theta, coords) with the coordinates standardised by the
    kept rows' column means and standard deviations (jws_column_stats, or the
    given `stats`), gathered in order by jws_gather_standardize.  Returns
    (X kept x 8, T kept x 2016, (mean, std))."""
    import torch
    rows = coords.shape[0]
    idx_h = np.nonzero(keep.cpu().numpy())[0].astype(np.int32)
    kept = len(idx_h)
    if stats is None:
        mean = torch.empty(NC, dtype=torch.float32, device="cuda")
        std = torch.empty(NC, dtype=torch.float32, device="cuda")
        work = torch.empty(int(jx.lib().jws_column_stats_work(rows, NC)) // 8 + 1, dtype=torch.float64,
                           device="cuda")
        _chk(jx.lib().jws_column_stats(rows, NC, _p(coords), _p(keep), kept, eps, _p(mean), _p(std), _p(work),
                                       _s()), "jws_column_stats")
    else:
        mean, std = stats
    idx = torch.from_numpy(idx_h).cuda()
    th = torch.as_tensor(theta, dtype=torch.float32, device="cuda").contiguous()
    X = torch.empty(kept, NIN, dtype=torch.float32, device="cuda")
    T = torch.empty(kept, NC, dtype=torch.float32, device="cuda")
    _chk(jx.lib().jws_gather_standardize(kept, _p(idx), NIN, _p(th), NC, _p(coords), _p(mean), _p(std), _p(X),
                                         _p(T), _s()), "jws_gather_standardize")
    return X, T, (mean, std)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
class Net:
    """FP32 master parameters, BF16 copy, Adam moments (device)."""

    def __init__(self, seed=0):
        import torch
        assert int(jx.lib().jws_param_count()) == NPARAM
        rng = np.random.default_rng(seed)
        p = np.zeros(NPARAM, dtype=np.float32)
        for off, fan_in, rows, cols in ((OFF_W1, NIN, NIN, HID), (OFF_W2, HID, HID, HID), (OFF_W3, HID, HID, NC)):
            lim = np.sqrt(6.0 / fan_in)   # He-uniform
            ld = cols
            w = rng.uniform(-lim, lim, size=(rows, cols)).astype(np.float32)
            p[off:off + rows * ld] = w.reshape(-1)
        self.master = torch.from_numpy(p).cuda()
        self.bf16 = torch.empty(NPARAM, dtype=torch.int16, device="cuda")
        self.grad = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
        self.m = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(NPARAM, dtype=torch.float32, device="cuda")
        self.step = 0
        self.mean = None
        self.std = None
        _chk(jx.lib().jws_to_bf16(NPARAM, _p(self.master), _p(self.bf16), _s()), "jws_to_bf16")
        self._acts = {}

    def acts(self, B):
        import torch
        if B not in self._acts:
            self._acts[B] = torch.empty(int(jx.lib().jws_acts_bytes(B)) // 2, dtype=torch.int16, device="cuda")
        return self._acts[B]

    def bias_ptr(self):
        return self.master.data_ptr() + 4 * OFF_B1

    def forward(self, theta, out=None):
        import torch
        B = theta.shape[0]
        out = torch.empty(B, NC, dtype=torch.float32, device="cuda") if out is None else out
        _chk(jx.lib().jws_mlp_forward(B, _p(theta), _p(self.bf16), self.bias_ptr(), _p(out), _p(self.acts(B)), _s()),
             "jws_mlp_forward")
        return out

    def backward(self, theta, dY):
        B = theta.shape[0]
        _chk(jx.lib().jws_mlp_backward(B, _p(self.acts(B)), _p(dY), _p(self.bf16), _p(self.grad),
                                       self.grad.data_ptr() + 4 * OFF_B1, _s()), "jws_mlp_backward")

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _chk(jx.lib().jws_adam_step(NPARAM, _p(self.master), _p(self.bf16), _p(self.grad), _p(self.m), _p(self.v),
                                    lr, b1, b2, eps, self.step, _s()), "jws_adam_step")

    def mse(self, Y, T, dY=None, loss=None):
        import torch
        loss = torch.empty(1, dtype=torch.float64, device="cuda") if loss is None else loss
        _chk(jx.lib().jws_mse(Y.shape[0], _p(Y), _p(T), _p(dY), _p(loss), _s()), "jws_mse")
        return loss


def train(net, theta, target, val_theta, val_target, epochs=40, batch=1024, lr=1e-3, patience=5, seed=1, log=None):
    """Adam with cosine-decayed learning rate on the MSE of standardised
    targets; early stop when the validation loss has not improved for
    `patience` epochs (the best parameters are kept)."""
    import torch
    m = theta.shape[0]
    steps_per_epoch = max(m // batch, 1)
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    dY = torch.empty(batch, NC, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    best, best_state, bad, hist = np.inf, None, 0, []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(m)).cuda()
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            th, tg = theta.index_select(0, idx), target.index_select(0, idx)
            Y = net.forward(th)
            net.mse(Y, tg, dY=dY, loss=loss)
            net.backward(th, dY)
            k = ep * steps_per_epoch + s
            net.adam(lr * 0.5 * (1.0 + np.cos(np.pi * k / total)))
        vl = float(net.mse(net.forward(val_theta), val_target).item())
        tl = float(loss.item())
        hist.append((ep, tl, vl))
        if log:
            log(f"epoch {ep}: train {tl:.4e} val {vl:.4e}")
        if not np.isfinite(best) or vl < best - 1e-6 * abs(best):
            best, bad = vl, 0
            best_state = (net.master.clone(), net.bf16.clone())
        else:
            bad += 1
            if bad >= patience:
                break
    torch.cuda.synchronize()
    if best_state is not None:
        net.master.copy_(best_state[0])
        net.bf16.copy_(best_state[1])
    return {"epochs": len(hist), "best_val": best, "history": hist, "seconds": time.perf_counter() - t0}


def propose(net, fam, theta):
    """Q0 (m x n x n, Q0[k] the matrix) for theta (m x 8 float32 CUDA)."""
    import torch
    m = theta.shape[0]
    Y = net.forward(theta)
    S = torch.empty(m, N, N, dtype=torch.float64, device="cuda")
    _chk(jx.lib().jws_skew_from_coords(m, N, _p(Y), _p(net.mean), _p(net.std), _p(S), _s()), "jws_skew_from_coords")
    Q0cm = torch.empty(m, N, N, dtype=torch.float64, device="cuda")
    _chk(jx.lib().jws_cayley_batched(m, N, _p(S), _p(fam.Qref_cm), _p(Q0cm), _s()), "jws_cayley_batched")
    return Q0cm.transpose(1, 2)   # column-major storage -> matrices


def generate(fam, count, seed, chunk=32768, log=None):
    """Thetas (count x 8, N(0, 0.1^2)), the solutions' canonical targets
    (count x 2016 FP32, CUDA) and the kept mask (int32, CUDA)."""
    import torch
    th = inputs.warmstart_thetas(count, seed)
    coords = torch.empty(count, NC, dtype=torch.float32, device="cuda")
    keep = torch.empty(count, dtype=torch.int32, device="cuda")
    for a in range(0, count, chunk):
        A = fam.matrices(th[a:a + chunk])
        _, Q, infos = solve(A)
        if (infos["status"] != 0).any():
            raise RuntimeError("training solve did not converge")
        c, k = canonical_targets(fam, Q)
        coords[a:a + chunk], keep[a:a + chunk] = c, k
        if log:
            log(f"generated {min(a + chunk, count)}/{count}")
    return th, coords, keep


def fixed_start(fam, m, mean=None, std=None):
    """Starts that use no network: Q0 = Qref for every matrix (mean None), or
    Q0 = Qref cay(S_mean) with S_mean the generator of the mean standardised
    target (coordinates 0 * std + mean, through the same kernels as the
    network's proposals)."""
    import torch
    if mean is None:
        return fam.Qref.unsqueeze(0).expand(m, N, N).contiguous()
    zero = torch.zeros(m, NC, dtype=torch.float32, device="cuda")
    S = torch.empty(m, N, N, dtype=torch.float64, device="cuda")
    _chk(jx.lib().jws_skew_from_coords(m, N, _p(zero), _p(mean), _p(std), _p(S), _s()), "jws_skew_from_coords")
    Q0cm = torch.empty(m, N, N, dtype=torch.float64, device="cuda")
    _chk(jx.lib().jws_cayley_batched(m, N, _p(S), _p(fam.Qref_cm), _p(Q0cm), _s()), "jws_cayley_batched")
    return Q0cm.transpose(1, 2)


def evaluate(net, fam, test_theta, reps=5):
    """Batched FP64 solves of the test batch from four starts: cold (Q0 = I),
    Qref for all, Qref cay(S_mean) (no network), and the network's proposal.
    Sweeps, their histograms, fallback rate and solves/s (median of `reps`
    timed calls; a start's own cost -- network, skew assembly, Cayley map --
    is inside its timed region)."""
    import torch
    A = fam.matrices(test_theta)
    th = torch.from_numpy(np.ascontiguousarray(test_theta, dtype=np.float32)).cuda()
    m = A.shape[0]

    def timed(fn):
        ts, r = [], None
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return r, float(np.median(ts[1:]))

    starts = {
        "cold": lambda: solve(A),
        "qref": lambda: solve(A, Q0=fixed_start(fam, m)),
        "mean_generator": lambda: solve(A, Q0=fixed_start(fam, m, net.mean, net.std)),
        "network": lambda: solve(A, Q0=propose(net, fam, th)),
    }
    out = {"matrices": m}
    ok = True
    cold_sweeps = None
    for name, fn in starts.items():
        (_, _, inf), t = timed(fn)
        sw = inf["sweeps"].astype(np.int64)
        if cold_sweeps is None:
            cold_sweeps = sw
        ok = ok and bool((inf["status"] == 0).all())
        out[name] = {"sweeps_mean": float(sw.mean()),
                     "sweeps_hist": {int(k): int(v) for k, v in zip(*np.unique(sw, return_counts=True))},
                     "sweeps_saved_mean": float((cold_sweeps - sw).mean()),
                     "fallback_rate": float(inf["fallback_used"].mean()), "solves_per_s": m / t, "seconds": t}
    out["status_ok"] = ok
    out["cold_sweeps_mean"] = out["cold"]["sweeps_mean"]
    out["warm_sweeps_mean"] = out["network"]["sweeps_mean"]
    out["speedup"] = out["network"]["solves_per_s"] / out["cold"]["solves_per_s"]
    out["speedup_vs_best_fixed_start"] = out["network"]["solves_per_s"] / max(
        out["qref"]["solves_per_s"], out["mean_generator"]["solves_per_s"])
    return out


def run(train_count=1 << 18, epochs=40, val_count=4096, test_count=4096, seed=5, log=print):
    fam = Family(seed)
    t0 = time.perf_counter()
    th, coords, keep = generate(fam, train_count, 50, log=log)
    gen_s = time.perf_counter() - t0
    vth, vco, vkeep = generate(fam, val_count, 51)
    X, T, stats = standardized(th, coords, keep)
    VX, VT, _ = standardized(vth, vco, vkeep, stats=stats)
    net = Net(seed=0)
    net.mean, net.std = stats
    dropped = 1.0 - X.shape[0] / train_count
    del coords
    tr = train(net, X, T, VX, VT, epochs=epochs, log=log)
    test_theta = inputs.warmstart_thetas(test_count, 52)
    ev = evaluate(net, fam, test_theta)
    return {"train_samples": int(train_count), "dropped_fraction": float(dropped),
            "generation_seconds": gen_s, "training": {k: v for k, v in tr.items() if k != "history"},
            "val_history": tr["history"], "test": ev}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=1 << 18)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run(a.train, a.epochs, log=lambda s: print(s, flush=True))
    txt = json.dumps(res, indent=1)
    print(txt)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)


if __name__ == "__main__":
    main()
