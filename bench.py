"""Benchmark: interval-SVD solves per second on one MI355X.

One "step" is one full ``csvd_solve_interval`` call (Algorithm 1: shifted
solves and moments, low-rank step, QR of A V~, SVD of B and the residual
check) on a synthetic sparse matrix already resident in HBM.

Default workload (--config c2): random sparse A, m = 200000, n = 100000, 10
nonzeros per column at uniform random rows, N(0,1) values, CSR FP64; the
interval holds about 64 singular values near the median of the spectrum
(located on a 25x smaller same-distribution instance); N = 32, L = 64,
M = 8, FP64.  --config c1 runs the 1200 x 1000 Givens-rotated matrix with
exactly known singular values on [0.40, 0.45] (N = 16, L = 16, M = 8).

Prints one JSON line (see the field list at the end of main()).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFS = 78.6  # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0

# DRAM-side bytes per launch of the two sparse products of the block step at
# c2, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB copy
# (FETCH x2.00, WRITE x1.00); valid only for the kernel source they were
# measured on (sha256 of csrc/k_bspmm.hip) and for the c2 workload.
SPMM_TRAFFIC_C2 = {"sha256": "a11d536573565865a171af39433ca82881a04271bcda9830f6b99ada4ad50863",
                   "bytes": (244868.0 * 2.0 + 100000.9 + 250765.6 * 2.0 + 50011.1) * 1024.0}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    import numpy as np
    import synth
    if name == "c1":
        I = synth.givens_known()
        return dict(I=I, a=I.a, b=I.b, L=16, M=8, N=16, ell=2, norm_a=1.0,
                    desc="givens_1200x1000_linspace_sigma_[0.40,0.45]")
    if name == "c2":
        m, n = 200000, 100000
        I = synth.random_sparse(m, n, 10, config=2)
        a, b, lq, dens = synth.interval_from_sample(m, n, 10, 64, config=2)
        return dict(I=I, a=a, b=b, L=64, M=8, N=32, ell=1, norm_a=0.0,
                    desc=f"random_sparse_{m}x{n}_10nnz_per_col_interval_64_near_median")
    raise SystemExit(f"unknown config {name}")


def cpu_baseline(W, iters_gpu, seconds=15.0):
    """The oracle's per-shift COCG (oracle/krylov.py, scipy CSR products) run
    for a bounded time on the full matrix, shift 1 of N/2, all L columns.
    One solve is extrapolated from the measured seconds per iteration times an
    iteration count: the larger of the Krylov dimension per column the GPU
    solve needed (its block steps) and the count the measured residual decay
    of the sample predicts for solve_rtol, times N/2 shifts and ell rounds."""
    import numpy as np
    import synth
    from oracle import krylov, quadrature as Q
    I = W["I"]
    shifts, c = Q.moment_coeffs(W["a"], W["b"], W["N"], W["M"], 0.1, Q.PLAIN)
    V = synth.v_in(I.n, W["L"], 2, 0)
    tol = W.get("solve_rtol", 1e-11)
    _, it, res, sec = krylov.cocg(I, shifts[0], V, tol=1e-300, maxit=10 ** 9, time_limit=seconds)
    per_it = sec / max(it, 1)
    worst = float(np.max(res)) if np.size(res) else 1.0
    rate = -np.log10(max(worst, 1e-300)) / max(it, 1)  # decades per iteration
    it_rate = int(np.ceil(-np.log10(tol) / rate)) if rate > 0 else None
    iters = max(iters_gpu, it_rate or 0)
    per_solve = per_it * iters * (W["N"] // 2) * W.get("ell", 1)
    threads = os.environ.get("OMP_NUM_THREADS", "unset")
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"oracle COCG (scipy CSR products, one thread) on shift 1 of {W['N'] // 2}, all {W['L']} "
                       f"columns of the full matrix: {it} iterations in {sec:.1f} s, worst relative residual "
                       f"{worst:.2e}; one solve = {per_it * 1e3:.1f} ms/iteration x {iters} iterations "
                       f"(max of the GPU block steps {iters_gpu} and the sample's decay rate "
                       f"{'%.2e' % rate} decades/iteration -> {it_rate}) x {W['N'] // 2} shifts x ell "
                       f"{W.get('ell', 1)} (extrapolated); OMP_NUM_THREADS={threads}")}


def spmm_traffic(config):
    import hashlib
    src = os.path.join(ROOT, "paper_2109_13655_amd", "csrc", "k_bspmm.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if config != "c2" or h != SPMM_TRAFFIC_C2["sha256"]:
        return None
    return SPMM_TRAFFIC_C2["bytes"]


def roofline(info, config):
    """The sparse products: the block solver's K1 (U = A Q_k) and K2
    (W = A^T U) together; the per-column solver's K2 (A^T product fused with
    the Lanczos update).  Algorithmic bytes per launch from the library
    (matrix + one read of the gathered block + the written block), times from
    HIP events recorded on the solve's stream around sampled launches."""
    if info.solver == 1:  # CSVD_SOLVER_BLOCK
        b = info.spmm_a_bytes + info.spmm_at_bytes
        t = info.spmm_a_ms + info.spmm_at_ms
        name = "b_spmm_a + b_spmm_at (U = A Q_k, W = A^T U on n x Lp blocks)"
    else:
        b, t = info.spmm_at_bytes, info.spmm_at_ms
        name = "k2_spmm_lanczos (A^T product + Lanczos update + window store)"
    ach = b / (t * 1e-3) / 1e9 if t > 0 else None
    traffic = spmm_traffic(config) if info.solver == 1 else None
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (ach / HBM_PEAK_GBS) if ach else None, "traffic": traffic,
            "bytes_per_launch": b, "avg_launch_ms": t, "samples": int(info.spmm_samples)}


def roofline_moments(info, W):
    """The moment accumulation of the block solver, S += [Q_k0 .. Q_k0+15]
    [F_k0; ..; F_k0+15] on FP64 MFMA: 2 n Lp (M + 1) L flops per basis block,
    16 blocks per launch, timed with HIP events around every full launch."""
    if info.solver != 1 or not info.moments_ms > 0:
        return None
    I = W["I"]
    Lp = int(info.L_padded)
    kmom = (W["M"] + 1) if W["ell"] == 1 else 1
    flops = 2.0 * I.n * Lp * kmom * W["L"] * 16
    ach = flops / (info.moments_ms * 1e-3) / 1e12
    return {"bound": "mfma", "kernel": "b_moments (S += Q F over 16 basis blocks)", "achieved": ach,
            "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFS, "traffic": None,
            "flops_per_launch": flops, "avg_launch_ms": info.moments_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--max-iters", type=int, default=0)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (a kernel of known traffic for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is single-GPU by design "
              "(shift sharding across GPUs is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2109_13655_amd as cs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    W = workload(args.config)
    I = W["I"]
    log("workload", W["desc"], "nnz", I.nnz, "interval", W["a"], W["b"])
    ctx = cs.csvd_create(I.m, I.n, I.rowptr, I.colidx, I.vals, hip_stream=stream.cuda_stream)
    p = cs.csvd_params_default(L=W["L"], M=W["M"], N=W["N"], ell=W["ell"], norm_a=W["norm_a"],
                               precision=cs.CSVD_MIXED if args.precision == "mixed" else cs.CSVD_FP64,
                               window=args.window)
    if args.max_iters:
        p.max_iters = args.max_iters
    import synth
    V = synth.v_in(I.n, W["L"], 2, 0)
    for i in range(args.warmup):
        cs.csvd_solve_interval(ctx, W["a"], W["b"], p, V)
        log("warmup", i, "done")
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status = []
    for i in range(args.steps):
        s0 = time.perf_counter()
        status.append(cs.csvd_solve_interval(ctx, W["a"], W["b"], p, V))
        lat.append(time.perf_counter() - s0)
        info = cs.csvd_get_info(ctx)
        log(f"step {i}: {lat[-1]:.3f}s status {status[-1]} iters {info.iterations_total} t_hat {info.t_hat} "
            f"rank {info.rank} sigma_s1 {info.sigma_s1:.3e} deflated {info.deflated} solver {info.solver} "
            f"max resid {info.max_triplet_resid:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = cs.csvd_get_info(ctx)
    sigma, _, _, resid = cs.csvd_get_triplets(ctx, I.m, I.n, want_vectors=False)
    cs.csvd_destroy(ctx)

    elapsed = t1 - t0
    value = args.steps / elapsed
    at_gbs = info.spmm_at_bytes / (info.spmm_at_ms * 1e-3) / 1e9 if info.spmm_at_ms > 0 else None
    a_gbs = info.spmm_a_bytes / (info.spmm_a_ms * 1e-3) / 1e9 if info.spmm_a_ms > 0 else None
    lat_ms = sorted(x * 1e3 for x in lat)

    def pct(q):
        return lat_ms[min(len(lat_ms) - 1, int(math.ceil(q * len(lat_ms))) - 1)]

    out = {
        "metric": "interval-SVD solves/sec + SpMM HBM GB/s at rel. residual <=1e-8; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": W["desc"], "m": I.m, "n": I.n, "nnz": I.nnz, "interval": [W["a"], W["b"]],
                   "N": W["N"], "L": W["L"], "M": W["M"], "ell": W["ell"], "precision": args.precision,
                   "window": info.window},
        "p50_ms": pct(0.5),
        "p99_ms": pct(0.99),
        "spmm_hbm_gbs": at_gbs,
        "spmm_a_gbs": a_gbs,
        "max_rel_residual": float(resid.max()) if resid.size else None,
        "t_hat": int(info.t_hat),
        "lanczos_steps": int(info.iterations_total),
        "solver": {1: "block", 2: "single"}.get(int(info.solver), str(info.solver)),
        "deflated": int(info.deflated),
        "one_pass_steps": int(info.one_pass_steps),
        "basis_stored": bool(info.basis_stored),
        "converged": bool(info.converged),
        "status": status,
        "phase_ms": {"solve": info.t_solve_ms, "lowrank": info.t_lowrank_ms, "qr": info.t_qr_ms,
                     "extract": info.t_extract_ms},
        "roofline": roofline(info, args.config),
        "roofline_moments": roofline_moments(info, W),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle COCG sample)")
        W["solve_rtol"] = p.solve_rtol
        out["cpu_baseline"] = cpu_baseline(W, int(info.iterations))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
