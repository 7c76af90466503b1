"""Benchmark: solved samples/s at 512^2 to relative residual 1e-10.

Workload: the finest MLMC level (512^2, coarse stage 256^2) of the 5-level
Darcy configuration - sigma^2 = 1, correlation length 0.2, 256 KL modes -
with 4096 samples of seeded synthetic KL coordinates. One step is the whole
hot path for all 4096 samples, with the inputs already in HBM:
  - KL synthesis on the matrix cores, exp and the injected coefficient pyramid;
  - the full-multigrid pass giving Q^c (256^2 stage) and Q^f (512^2 stage),
    both driven to ||b - A p|| <= 1e-10 ||b||;
  - the compensated estimator reduction.
Forms: FP32 V-cycles + FP64 iterative refinement (headline `value`) and
plain FP64 FMG, each timed on the same samples.

Prints one JSON line (rank 0, N = 1). Multi-GPU runs are not part of this
build: --gpus > 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CFG = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=5, n0=32)
LEVEL = 4
N = 512
METRIC = "solved samples/s at 512² to rel-res 1e-10: FP32+IR/NN-warm vs FP64 FMG"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(torch, fmgmc, xi_dev, solver, args):
    S = xi_dev.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros_like(qf)
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    ctx = fmgmc.Context(**CFG, solver=solver, rel_tol=args.tol, max_batch=args.batch,
                        inner_cycles=args.inner, max_cycles=60)

    def step():
        rc = ctx.solve_level(LEVEL, xi_dev, qf, qc, cyc, fl)
        est = fmgmc.estimate([qf], [qc])
        return rc, est

    for w in range(args.warmup):
        step()
        log(f"[{solver}] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        rc, est = step()
        log(f"[{solver}] step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    prof = ctx.profile_read()
    ctx.close()
    dt = (t1 - t0) / args.steps
    c = cyc.cpu().numpy()
    return dict(samples_per_s=S / dt, ms_per_step=1e3 * dt, rc=int(rc),
                cycles_coarse_mean=float(c[:, 0].mean()), cycles_fine_mean=float(c[:, 1].mean()),
                cycles_fine_max=int(c[:, 1].max()), flags=int(fl.cpu().numpy().astype(np.int64).sum()),
                estimate=dict(mean_y=est["levels"][0]["mean_y"], var_y=est["levels"][0]["var_y"]),
                prof=prof, qf=qf.cpu().numpy(), qc=qc.cpu().numpy())


# Measured HBM traffic / algorithmic bytes of the dominant kernels, from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE passes calibrated on a plain 1 GiB copy
# (profiles/hbm_traffic_512.md). None once a kernel changes after measurement.
TRAFFIC_RATIO = {"ir": 1.000, "post": 1.000, "pre": 1.000}


def roofline(form, steps):
    """Dominant HBM-bound kernel of a form from the library's event timing."""
    best = None
    for kind in ("pre", "post", "ir"):
        ms, n, alg = form["prof"][kind]
        if n and (best is None or ms > best[1]):
            best = (kind, ms, n, alg)
    kind, ms, n, alg = best
    gbs = alg / (ms * 1e-3) / 1e9
    ratio = TRAFFIC_RATIO.get(kind)
    traffic = None if ratio is None else round(ratio * alg / n / 1e9, 4)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "GB per launch",
            "kernel": kind, "avg_launch_us": round(1e3 * ms / n, 2), "launches": n,
            "alg_bytes_per_launch": alg / n}


def cpu_baseline(xi, n_samples):
    from oracle import oracle as O
    threads = O.max_threads()
    tab = O.kl_table(CFG["sigma2"], CFG["corr_len"], CFG["n_modes"])
    sub = xi[:n_samples]
    t0 = time.perf_counter()
    O.solve_level(CFG["sigma2"], CFG["corr_len"], tab, N, LEVEL, sub, tol=1e-10, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(n_samples / dt, 3), "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_samples} of the 4096 samples at 512^2 (FP64 KL + FMG to 1e-10), "
                      f"{dt:.1f} s wall on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--inner", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--forms", default="fp32_ir,fp64")
    ap.add_argument("--cpu-samples", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the method's samples are independent; "
              "multi-GPU sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_04727_amd import fmgmc, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst
    xi = inputs.mc_normals(args.samples, CFG["n_modes"], config=2, level=LEVEL)
    xi_dev = torch.from_numpy(xi).to("cuda")
    torch.cuda.synchronize()

    forms = {}
    for solver in args.forms.split(","):
        log(f"form {solver}: {args.samples} samples at {N}^2, batch {args.batch}")
        forms[solver] = run_form(torch, fmgmc, xi_dev, solver, args)
        f = forms[solver]
        log(f"  {f['samples_per_s']:.1f} samples/s, {f['ms_per_step']:.1f} ms/step, cycles "
            f"{f['cycles_coarse_mean']:.2f}/{f['cycles_fine_mean']:.2f}, rc {f['rc']}")
    head = "fp32_ir" if "fp32_ir" in forms else list(forms)[0]
    H = forms[head]
    out = {
        "metric": METRIC, "value": round(H["samples_per_s"], 2), "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(H["ms_per_step"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if head == "fp32_ir" else "f64",
        "data": "synthetic (seeded PCG64 KL coordinates)",
        "config": {"workload": f"finest MLMC level {N}^2 (coarse stage {N // 2}^2) of the 5-level config, "
                               f"sigma2=1, corr_len=0.2, 256 KL modes, {args.samples} samples, "
                               f"rel-res {args.tol:g}, form {head}",
                   "batch": args.batch, "inner_cycles": args.inner},
        "roofline": roofline(H, args.steps),
    }
    out["forms"] = {}
    for k, f in forms.items():
        kl_ms, kl_n, kl_flops = f["prof"]["kl"]
        out["forms"][k] = {
            "samples_per_s": round(f["samples_per_s"], 2), "ms_per_step": round(f["ms_per_step"], 2),
            "cycles_coarse_mean": round(f["cycles_coarse_mean"], 3),
            "cycles_fine_mean": round(f["cycles_fine_mean"], 3), "cycles_fine_max": f["cycles_fine_max"],
            "status": f["rc"], "flagged_samples": f["flags"], "mean_Y": f["estimate"]["mean_y"],
            "roofline": roofline(f, args.steps),
            "kl_tflops": round(kl_flops / (kl_ms * 1e-3) / 1e12, 2) if kl_n else None,
        }
    if "fp32_ir" in forms and "fp64" in forms:
        a, b = forms["fp32_ir"], forms["fp64"]
        out["forms"]["ir_vs_fp64_speedup"] = round(a["samples_per_s"] / b["samples_per_s"], 3)
        out["forms"]["ir_vs_fp64_max_rel_qf_diff"] = float(np.max(np.abs(a["qf"] - b["qf"]) / np.abs(b["qf"])))
    if not args.no_cpu:
        log(f"cpu baseline: oracle on {args.cpu_samples} samples")
        out["cpu_baseline"] = cpu_baseline(xi, args.cpu_samples)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
