"""Benchmark of the batched safety filter on one MI355X.

One step = one sf_project call over the whole workload (every sample, every iteration,
final residual), inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FEAS_TOL = 1e-3          # m, m/s, m/s^2 at the grid times, checked in FP64
PEAKS = {                # published MI355X peaks
    "fp32_vector_tflops": 157.3,
    "bf16_mfma_tflops": 2500.0,
    "fp16_mfma_tflops": 2500.0,
    "fp32_mfma_tflops": 157.3,
    "fp64_vector_tflops": 78.6,
    "hbm_gbs": 8000.0,
}


def flops_per_sample_iter(cfg):
    """Algorithmic flops of one iteration for one sample (multiply-add = 2), counted as
    basis evaluation 6nDHm, back-projection to the free coefficients 6nDHm_f, the Gram
    product 4nDm m_f, pair projections 15 N_p H, bound balls 24nH, the pair scatter
    2 N_p H D, the multiplier/target update 5nDm_f and the QP product 2D(n m_f)^2."""
    n, D, m, H = cfg.n_robots, cfg.dims, cfg.degree + 1, cfg.horizon
    mf = m - 6
    Np = n * (n - 1) // 2
    return (6 * n * D * H * m + 6 * n * D * H * mf + 4 * n * D * m * mf + 15 * Np * H + 24 * n * H
            + 2 * Np * H * D + 5 * n * D * mf + 2 * D * (n * mf) ** 2)


def cpu_baseline(workload, n_samples, iters):
    """The FP64 oracle on a bounded sample of the same workload, on the host cores."""
    import torch
    import oracle as O
    p = workload.problems[0]
    s = O.build_system(p.cfg)
    xb = torch.tensor(p.xi_bar[:n_samples])
    bv = torch.tensor(p.bvals)
    t0 = time.perf_counter()
    O.sf_project(s, xb, bv, iters)
    dt = time.perf_counter() - t0
    return {"value": n_samples / dt, "unit": "projections/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"first {n_samples} of {p.xi_bar.shape[0]} samples, {iters} iterations, "
                      f"FP64 torch CPU ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="swarm16", choices=["swarm16", "swarm32", "tiny2d"])
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--cpu-samples", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--generic", action="store_true", help="force the generic (non-MFMA) kernel")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 3 device copies of 256 MiB (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; --gpus above 1 is not supported "
                                   "(samples shard across GPUs without communication, see the design notes)"}))
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2501_19042_amd import SafetyFilter

    torch.cuda.set_device(0)
    wl = W.WORKLOADS[args.workload]()
    p = wl.problems[0]
    prec = args.precision
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = SafetyFilter([p.cfg])
    xb = torch.tensor(p.xi_bar, dtype=dt, device="cuda")
    bv = torch.tensor(p.bvals, dtype=dt, device="cuda")
    S = xb.shape[0]
    K = wl.iters

    for _ in range(args.warmup):
        out = sf.project(xb, bv, K, precision=prec, generic=args.generic)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        out = sf.project(xb, bv, K, precision=prec, generic=args.generic)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps

    viol = sf.feasibility(out.xi, bv, precision=prec).cpu()
    feas = (viol[:, :3] <= FEAS_TOL).all(1) & (viol[:, 3] <= FEAS_TOL)
    n_conv = int(feas.sum())
    value = n_conv / (ms / 1e3)

    W_it = flops_per_sample_iter(p.cfg)
    flops = W_it * S * K
    achieved = flops / (ms / 1e3) / 1e12
    peak = PEAKS["fp64_vector_tflops"] if prec == "fp64" else PEAKS["fp32_vector_tflops"]
    line = {
        "metric": "converged SF projections/sec (16 robots, 3D); BF16-MFMA vs FP32 at equal residual",
        "value": round(value, 1),
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16+f32", "fp16": "f16+f32"}[prec],
        "data": "synthetic (seeded straight-line Bernstein fits + Gaussian coefficient noise)",
        "config": {"workload": wl.name, "samples": S, "robots": p.cfg.n_robots, "dims": p.cfg.dims,
                   "degree": p.cfg.degree, "horizon": p.cfg.horizon, "iters": K, "precision": prec,
                   "kernel": "generic" if args.generic else "mfma"},
        "converged_fraction": n_conv / S,
        "all_samples_per_s": round(S / (ms / 1e3), 1),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "flops_per_sample_iter": W_it, "kernel_ms": round(ms, 4)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_samples, S), K)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
