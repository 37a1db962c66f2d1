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


def hbm_probe(torch, gib=2):
    """Plain-kernel HBM ceilings on this GPU: a device copy and a read-only reduction
    of 2 GiB (best of 5 each), for context next to the 8 TB/s peak."""
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best_c = best_r = 1e9
    for _ in range(5):
        e0.record(); b.copy_(a); e1.record(); torch.cuda.synchronize()
        best_c = min(best_c, e0.elapsed_time(e1))
        e0.record(); a.sum(); e1.record(); torch.cuda.synchronize()
        best_r = min(best_r, e0.elapsed_time(e1))
    del a, b
    return {"copy_gbs": round(2 * n * 8 / best_c / 1e6, 1), "read_gbs": round(n * 8 / best_r / 1e6, 1),
            "bytes": n * 8}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("dslash.hip", "device_common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_0710_0066_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(prec):
    """HBM bytes per hop launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by
    a plain copy of known size) for the hop kernel source it was taken on; None when the
    kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", "hop_traffic_24x24x24x48.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    entry = rec.get(prec)
    return None if entry is None else entry["traffic_bytes_per_launch"]


def block_solve_comparison(sap, torch, ctx, cfg, L, repeats=3):
    """Wall time (call to verified return) of the batched block solves of the 24^3x48
    workload: level 1 (12 blocks of 24^3x4) and level 2 (24 blocks of 24^3x2), 12
    Gaussian right-hand sides each, to ||b - W x|| / ||b|| <= 1e-10 recomputed in FP64.
    mixed = FP32 inner solves inside the FP64 defect correction, all systems batched;
    fp64 = FP64 inner solve, all systems batched; fp64_rhs_loop = FP64, one right-hand
    side per call (the blocks of a level are always solved together)."""
    import numpy as np
    import synth
    nrhs = cfg["nrhs"]
    b = synth.gaussian_spinor(L, cfg["seed_src"], nrhs=nrhs)
    fb = ctx.new_field(nrhs)
    ctx.pack_spinor(fb, torch.from_numpy(b).cuda(), nrhs)
    del b
    fx = ctx.new_field(nrhs)
    one = ctx.field_bytes(1) // 8
    mixed = sap.solve_opts(tol=1e-10, inner_prec=sap.SAP_F32, inner_tol=1e-5)
    plain = sap.solve_opts(tol=1e-10, inner_prec=sap.SAP_F64, inner_tol=0.0)

    def run(opts, per_rhs):
        ts, worst, iters = [], 0.0, 0
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = []
            for level in (1, 2):
                if per_rhs:
                    for r in range(nrhs):
                        infos += sap.solve_blocks(ctx, fx[r * one:(r + 1) * one], fb[r * one:(r + 1) * one],
                                                  1, level, sap.SAP_ALL, opts)
                else:
                    infos += sap.solve_blocks(ctx, fx, fb, nrhs, level, sap.SAP_ALL, opts)
            ts.append(time.perf_counter() - t0)
            worst = max(e.true_rel_res for e in infos)
            iters = max(e.iters for e in infos)
        return {"seconds": float(np.median(ts)), "max_true_rel_res": worst, "max_iters": iters}

    print("[bench] block solves: mixed batched", file=sys.stderr, flush=True)
    m = run(mixed, False)
    print("[bench] block solves: fp64 batched", file=sys.stderr, flush=True)
    f = run(plain, False)
    print("[bench] block solves: fp64 one rhs per call", file=sys.stderr, flush=True)
    fl = run(plain, True)
    return {"systems": f"{nrhs} rhs x (12 blocks 24^3x4 + 24 blocks 24^3x2) = {nrhs * 36}",
            "tol": 1e-10, "mixed_batched": m, "fp64_batched": f, "fp64_rhs_loop": fl,
            "speedup_vs_fp64_batched": f["seconds"] / m["seconds"],
            "speedup_vs_fp64_rhs_loop": fl["seconds"] / m["seconds"]}


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
        # plain device copy of 1 GiB whose source was pushed out of the 256 MB MALL by a
        # second 1 GiB fill: the counters of this copy read 1 GiB fetched, 1 GiB written
        n = 1024 * 1024 * 1024 // 8
        a = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
        c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b, c
        print(f"[bench] copy calibration: one copy of {n * 8} bytes", file=sys.stderr, flush=True)

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

    if not args.only_dslash:
        result["hbm_probe"] = hbm_probe(torch)

    traffic = committed_traffic(args.prec)
    if traffic is not None:
        result["roofline"]["traffic"] = traffic

    if not args.only_dslash and not args.skip_solve:
        result["block_solve"] = block_solve_comparison(sap, torch, ctx, cfg, L)

    if not args.only_dslash and not args.skip_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(U, psi, k, V, args.prec)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
