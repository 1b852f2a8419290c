#!/usr/bin/env python3
"""Benchmark of the blocked Jacobi eigensolver on one MI355X.

Main line (the headline workload): blocked two-sided Jacobi eigendecomposition,
n = 4096, b = 64 (64 block columns, 32 block pairs per parallel step), graded
spectrum lambda_i = +-10^(-8 i / n) (Haar Q, seed 2), FP64, to
Xi(A) <= 1e-14 ||A||_F, with eigenvectors and orthogonality refinement.  One
step = one full solve (jacobi_eig) on inputs already resident in HBM.

Reported beside it on the same JSON line:
  * roofline: the dominant kernel's algorithmic flops per launch over its
    average launch time, timed with HIP events the library records on the
    launch stream during the timed steps; `traffic` from the committed
    rocprofv3 counter summary when it was taken on the current kernel source;
  * cpu_baseline: the CPU oracle (scalar FP64 round-robin Jacobi, all host
    cores) on a bounded sample of the same matrix, scaled to s/solve;
  * extras: the batched workload (10,000 matrices, n ~ U{16..256}, FP32
    stored, to 1e-12 residuals) in solves/s against per-matrix plain FP64
    calls, the FP32 precision ladder on the headline matrix, and the one-sided
    SVD of 16384 x 2048 (sigma log-uniform in [1e-6, 1]).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]
    python bench.py --copy-probe MiB     # plain copy kernel of known size (counter scaling)
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "block-Jacobi eig n=4096 s/solve & %MFMA peak; batched solves/s vs plain @1e-12"
N = 4096
BLOCK = 64
SEED = 2
PEAK = {"fp64_tflops": 78.6, "hbm_gbs": 8000.0}
KINDS = {0: "k_subproblem2", 1: "k_update_a_crit", 2: "k_update_q", 3: "k_gemm_f64", 5: "k_update_a_bounded",
         6: "k_update_aq_bounded"}
SOURCES = {"k_subproblem2": ["k_subproblem.hip", "jx_sweep.hpp"], "k_update_a_crit": ["k_update.hip"],
           "k_update_q": ["k_update.hip"], "k_gemm_f64": ["k_gemm.hip"], "k_update_a_bounded": ["k_update.hip"],
           "k_update_aq_bounded": ["k_update.hip"]}
# kernels on the second stream, beside the next round's subproblems (not on
# the solve's critical path): not candidates for the dominant kernel
SIDE = {"k_update_q", "k_update_a_bounded", "k_update_aq_bounded"}


def kernel_source_hash(name):
    h = hashlib.sha256()
    for src in SOURCES[name]:
        with open(os.path.join(ROOT, "paper_2608_28952_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/<kernel>_n4096_b64_traffic.md, lines `key: value`), if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{name}_n4096_b64_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip().lstrip("-* ").strip("`")] = v.strip().strip("`")
    if kv.get("source_sha256_16") != kernel_source_hash(name):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(A, gpu_sweeps, target_s=20.0):
    """The oracle (scalar round-robin Jacobi, FP64, all host cores) on the same
    matrix: k round-robin rounds of sweep 1, k chosen for about target_s
    seconds.  The time of a 1-round run (the oracle's setup: copies, Q = I,
    off-norms, sorting, plus one round) is subtracted, so the figure is the
    rotation rate, scaled to s/solve as (time per rotation) x n(n-1)/2
    rotations per sweep x the GPU's sweep count."""
    from oracle import oracle as O
    cores = os.cpu_count() or 1
    n = A.shape[0]

    def run(rounds):
        t0 = time.perf_counter()
        r = O.eig(A, order=1, nthreads=cores, max_rotations=rounds * (n // 2), max_sweeps=1)
        return time.perf_counter() - t0, r.rotations

    t1, r1 = run(1)
    t8, r8 = run(8)
    per_round = max((t8 - t1) / 7.0, 1e-6)
    k = int(min(n - 1, max(9, target_s / per_round)))
    tk, rk = run(k)
    dt, drot = tk - t1, rk - r1
    per_rot = dt / max(drot, 1)
    return {"value": per_rot * n * (n - 1) / 2 * gpu_sweeps, "unit": "s/solve", "cores": cores, "kind": "oracle",
            "seconds_measured": dt,
            "sample": (f"{drot} rotations ({k} minus 1 round-robin rounds of sweep 1, the 1-round run's time, "
                       f"{t1:.2f} s of it setup, subtracted) on the same n={n} matrix in {dt:.1f} s, scaled by "
                       f"n(n-1)/2 rotations per sweep x {gpu_sweeps} sweeps (the GPU solve's sweep count)")}


def copy_probe(mib, reps=20):
    """A plain device copy of `mib` MiB, `reps` times (reads and writes mib MiB
    each): the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "reps": reps, "bytes_read_per_launch": n * 8,
                      "bytes_written_per_launch": n * 8}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def extras(jx):
    import torch
    from paper_2608_28952_amd import inputs
    out = {}
    log("extras: batched workload")
    # batched workload against per-matrix plain FP64 calls
    sizes, offs, packed = inputs.batched_case(10000, 4)
    o = jx.opts_default(precision=jx.PREC_MIXED_FP32)
    dA = torch.from_numpy(packed).cuda()
    ws = torch.empty(jx.batched_workspace(sizes, False, o), dtype=torch.uint8, device="cuda")
    W = torch.empty(int(sizes.sum()), dtype=torch.float64, device="cuda")
    Q = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    times = []
    for _ in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, infos = jx.jacobi_eig_batched(sizes, offs, dA, opts=o, work=ws, out=(W, Q), info="array")
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ok = bool((infos["status"] == 0).all())
    tb = float(np.median(times[1:]))
    idx = np.random.default_rng(0).choice(len(sizes), 40, replace=False)
    tp = 0.0
    for k in idx:
        n = int(sizes[k])
        A = torch.from_numpy(np.ascontiguousarray(packed[offs[k]:offs[k + 1]].astype(np.float64)
                                                  .reshape((n, n), order="F"))).cuda()
        jx.jacobi_eig(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        jx.jacobi_eig(A)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
    plain = len(idx) / tp
    out["batched"] = {"workload": "10,000 symmetric matrices, n ~ U{16..256}, lambda ~ N(0,1), FP32 stored, seed 4; "
                                  "FP32 phase + FP64 refinement to off(A) <= 1e-14 ||A||_F, one cached hipGraph launch",
                      "solves_per_s": len(sizes) / tb, "ms_per_batch": tb * 1e3, "all_converged": ok,
                      "max_off_rel": float(infos["off_rel"].max()),
                      "fp32_sweeps_mean": float(infos["sweeps_by_prec"][:, 1].mean()),
                      "fp64_sweeps_mean": float(infos["sweeps_by_prec"][:, 2].mean()),
                      "plain_fp64_per_matrix_solves_per_s": plain,
                      "plain_sample": "40 matrices of the batch, one jacobi_eig call each (FP64)",
                      "speedup_vs_plain": (len(sizes) / tb) / plain}
    del dA, ws, W, Q
    log("extras: FP32 ladder n=4096")
    # FP32 ladder on the headline matrix
    A_np, lam = inputs.eig_graded(N, SEED)
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    om = jx.opts_default(block=BLOCK, precision=jx.PREC_MIXED_FP32)
    work = torch.empty(jx.jacobi_eig_workspace(N, om), dtype=torch.uint8, device="cuda")
    jx.jacobi_eig(A, opts=om, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Wm, Qm, info = jx.jacobi_eig(A, opts=om, work=work)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    out["mixed_fp32_eig_n4096"] = {"s_per_solve": tm, "sweeps_by_prec": info["sweeps_by_prec"],
                                   "max_abs_eig_err_vs_construction":
                                       float(np.max(np.abs(Wm.cpu().numpy() - np.sort(lam))))}
    del A, work
    log("extras: SVD 16384 x 2048")
    # one-sided SVD, FP64 and FP32 ladder
    G_np, sigma = inputs.svd_case(16384, 2048, 3)
    G = torch.from_numpy(np.ascontiguousarray(G_np)).cuda()
    ref = np.sort(sigma)[::-1]
    for name, prec in (("svd_16384x2048_fp64", jx.PREC_FP64), ("svd_16384x2048_mixed_fp32", jx.PREC_MIXED_FP32)):
        os_ = jx.opts_default(precision=prec)
        jx.jacobi_svd(G, opts=os_)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S, U, V, info = jx.jacobi_svd(G, opts=os_)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        Sn = S.cpu().numpy()
        out[name] = {"s_per_solve": ts, "sweeps_by_prec": info["sweeps_by_prec"],
                     "max_rel_sigma_err_vs_construction": float(np.max(np.abs(Sn - ref) / ref))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU and is measured on one GPU only "
              f"(got --gpus {args.gpus}); a sharding over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import torch
    from paper_2608_28952_amd import inputs
    from paper_2608_28952_amd import jacobi as jx

    A_np, lam = inputs.eig_graded(N, SEED)
    A = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    o = jx.opts_default(block=BLOCK)
    work = torch.empty(jx.jacobi_eig_workspace(N, o), dtype=torch.uint8, device="cuda")
    L = jx.lib()

    log(f"warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        jx.jacobi_eig(A, opts=o, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        W, Q, info = jx.jacobi_eig(A, opts=o, work=work)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel HIP events (library profiler) over a second pass of the same
    # steps: the events and the per-round flag copies that price the
    # subproblem work cost time of their own, so `value` comes from the pass
    # above, which runs without them
    log("profiled pass")
    L.jacobi_profile_enable(1)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        jx.jacobi_eig(A, opts=o, work=work)
    torch.cuda.synchronize()
    prof = {}
    for k, name in KINDS.items():
        cnt, ms, fl, by = ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        L.jacobi_profile_query(k, ctypes.byref(cnt), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by))
        prof[name] = {"launches": cnt.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
    L.jacobi_profile_enable(0)

    sec = (t1 - t0) / args.steps
    W_np = W.cpu().numpy()
    err = float(np.max(np.abs(W_np - np.sort(lam))))
    sweeps = infos[-1]["sweeps"]

    dom = max((k for k in prof if k not in SIDE), key=lambda k: prof[k]["ms"])
    d = prof[dom]
    launches = max(d["launches"], 1)
    avg_s = d["ms"] / 1e3 / launches
    ach = d["flops"] / launches / avg_s / 1e12
    bound = "alu" if dom == "k_subproblem2" else "mfma"
    roof = {"bound": bound, "achieved": ach, "peak": PEAK["fp64_tflops"], "unit": "TFLOP/s",
            "frac": ach / PEAK["fp64_tflops"], "traffic": None,
            "kernel": dom, "avg_launch_us": avg_s * 1e6, "launches": d["launches"],
            "algorithmic_flops_per_launch": d["flops"] / launches}
    t = traffic_for(dom)
    if t is not None:
        roof["traffic"] = t
    # whole-solve rate: Alg. 2's rotation-apply work per sweep, 12 n^2 b (N - 1)
    # flops (both block rows and block columns of A, and Q), over the solve time
    nb = N // BLOCK
    f_sweep = 12.0 * N * N * BLOCK * (nb - 1)
    solve_rate = {"flops_per_sweep": f_sweep, "tflops": f_sweep * sweeps / sec / 1e12,
                  "frac_of_fp64_peak": f_sweep * sweeps / sec / 1e12 / PEAK["fp64_tflops"]}
    others = {k: {"avg_launch_us": v["ms"] * 1e3 / max(v["launches"], 1), "launches": v["launches"],
                  "achieved_tflops": (v["flops"] / max(v["ms"], 1e-12) / 1e9) if v["ms"] > 0 else 0.0}
              for k, v in prof.items()}
    total_ms = sum(x["ms"] for x in prof.values())
    share = {k: round(v["ms"] / max(total_ms, 1e-9), 4) for k, v in prof.items()}

    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "blocked two-sided Jacobi eig, n=4096, b=64 (32 block pairs per parallel step), "
                               "graded spectrum +-10^(-8i/n), Haar Q seed 2, FP64, off(A) <= 1e-14 ||A||_F, "
                               "eigenvectors + orthogonality refinement",
                   "n": N, "block": BLOCK, "sweeps": sweeps, "max_abs_eig_err_vs_construction": err,
                   "kernel_time_share": share, "kernels": others, "solve_rotation_apply_rate": solve_rate},
        "roofline": roof,
    }
    log(f"{sec:.3f} s/solve, {sweeps} sweeps")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(A_np, sweeps)
    if not args.no_extras:
        del A, work
        torch.cuda.empty_cache()
        out["extras"] = extras(jx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
