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
import math
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


WEIGHTS = os.path.join(ROOT, "paper_1910_04727_amd", "weights", "cnn_cfg2.bin")


def run_form(torch, fmgmc, xi_dev, form, args, tol=None, steps=None, warmup=None, separate_coarse=False):
    """form: fp32_ir, fp64, or nn_warm (fp32_ir whose QoI stages with warm_min_n <= n <= warm_max_n start
    from the trained network: by default the 256^2 stage).
    tol / steps / warmup default to the command line's; separate_coarse: the standard-MLMC
    comparator (Q^c from its own FMG solve on 256^2)."""
    tol = args.tol if tol is None else tol
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    solver = "fp32_ir" if form == "nn_warm" else form
    S = xi_dev.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros_like(qf)
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    nu1, nu2 = (int(v) for v in args.nu.split(",")) if solver == "fp32_ir" else (2, 2)
    ctx = fmgmc.Context(**CFG, solver=solver, rel_tol=tol, max_batch=args.batch,
                        inner_cycles=args.inner, max_cycles=60, nu1=nu1, nu2=nu2, w_max_n=args.wmax,
                        inner_first=args.inner_first, fuse_cycles=not args.no_fuse,
                        separate_coarse=separate_coarse)
    net = None
    if form == "nn_warm":
        net = fmgmc.Cnn(path=WEIGHTS)
        ctx.set_warm_start(net, min_n=args.warm_min_n, max_n=args.warm_max_n)

    def step():
        rc = ctx.solve_level(LEVEL, xi_dev, qf, qc, cyc, fl)
        est = fmgmc.estimate([qf], [qc])
        return rc, est

    tag = f"{form} tol {tol:g}" + (" separate coarse" if separate_coarse else "")
    for w in range(warmup):
        step()
        log(f"[{tag}] warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for k in range(steps):
        rc, est = step()
        log(f"[{tag}] step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    prof = ctx.profile_read()
    ctx.close()
    if net is not None:
        net.close()
    dt = (t1 - t0) / steps
    c = cyc.cpu().numpy()
    return dict(samples_per_s=S / dt, ms_per_step=1e3 * dt, rc=int(rc),
                cycles_coarse_mean=float(c[:, 0].mean()), cycles_fine_mean=float(c[:, 1].mean()),
                cycles_fine_max=int(c[:, 1].max()), flags=int(((fl.cpu().numpy() & 7) != 0).sum()),
                warm_rejected=int(((fl.cpu().numpy() & fmgmc.FLAG_WARM_REJECTED) != 0).sum()),
                estimate=dict(mean_y=est["levels"][0]["mean_y"], var_y=est["levels"][0]["var_y"]),
                prof=prof, qf=qf.cpu().numpy(), qc=qc.cpu().numpy(), cycles=c)


# Measured HBM traffic / algorithmic bytes of the dominant kernels, from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE passes calibrated on a plain 1 GiB copy
# (profiles/hbm_traffic_512.md; taken offline, not in this run). None once a
# kernel changes after measurement.
TRAFFIC_RATIO = {"ir": None, "post": 1.000, "pre": 1.000, "fused": 1.000, "irpre": 1.000}
TRAFFIC_SOURCE = ("rocprofv3 FETCH_SIZE / WRITE_SIZE passes over the same launch, calibrated on a plain "
                  "copy (profiles/hbm_traffic_512.md); taken offline, not in this run")
STENCIL_TARGET = 0.60  # fraction of the HBM peak the stencil passes aim for


def roofline(form, steps):
    """Dominant HBM-bound kernel of a form from the library's event timing."""
    best = None
    for kind in ("pre", "post", "ir", "fused", "irpre"):
        ms, n, alg = form["prof"][kind]
        if n and (best is None or ms > best[1]):
            best = (kind, ms, n, alg)
    kind, ms, n, alg = best
    gbs = alg / (ms * 1e-3) / 1e9
    ratio = TRAFFIC_RATIO.get(kind)
    traffic = None if ratio is None else round(ratio * alg / n / 1e9, 4)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "GB per launch",
            "traffic_source": TRAFFIC_SOURCE if traffic is not None else None,
            "kernel": kind, "avg_launch_us": round(1e3 * ms / n, 2), "launches": n,
            "alg_bytes_per_launch": alg / n,
            "stencil_passes_512": pass_table(form),
            "stencil_passes_below_target": sorted(k for k, v in pass_table(form).items()
                                                  if v["frac"] < STENCIL_TARGET)}


def pass_table(form):
    """Per-kind figures of the three timed 512^2 stage passes: launches, mean
    launch time and algorithmic GB/s (the roofline picks the largest total)."""
    out = {}
    for kind in ("pre", "post", "ir", "fused", "irpre"):
        ms, n, alg = form["prof"][kind]
        if n:
            gbs = alg / (ms * 1e-3) / 1e9
            out[kind] = {"launches": n, "avg_launch_us": round(1e3 * ms / n, 2),
                         "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def cpu_baseline(xi, n_samples, tol, wmax):
    """The oracle timed on the host cores on the first n_samples samples; also
    returns its Q^f, Q^c and cycle counts (the reference of the accuracy records)."""
    from oracle import oracle as O
    threads = O.max_threads()
    tab = O.kl_table(CFG["sigma2"], CFG["corr_len"], CFG["n_modes"])
    sub = xi[:n_samples]
    t0 = time.perf_counter()
    oqf, oqc, ocyc, _ = O.solve_level(CFG["sigma2"], CFG["corr_len"], tab, N, LEVEL, sub, tol=tol,
                                      nthreads=threads, wmax=wmax)
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(n_samples / dt, 3), "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_samples} of the 4096 samples at 512^2 (FP64 KL + FMG to {tol:g}), "
                      f"{dt:.1f} s wall on {threads} threads",
            "cpu_model": model, "host_cpus": os.cpu_count()}, (oqf, oqc, ocyc)


def oracle_ref(xi, n_samples, tol, wmax):
    """Oracle Q^f, Q^c on the first n_samples samples (untimed reference)."""
    from oracle import oracle as O
    tab = O.kl_table(CFG["sigma2"], CFG["corr_len"], CFG["n_modes"])
    oqf, oqc, ocyc, _ = O.solve_level(CFG["sigma2"], CFG["corr_len"], tab, N, LEVEL, xi[:n_samples], tol=tol,
                                      nthreads=O.max_threads(), wmax=wmax)
    return oqf, oqc, ocyc


def qoi_err(form, ref):
    """Per-sample relative QoI error of a form against the oracle on the reference samples."""
    oqf, oqc, ocyc = ref
    k = len(oqf)
    ef = np.abs(form["qf"][:k] - oqf) / np.abs(oqf)
    ec = np.abs(form["qc"][:k] - oqc) / np.abs(oqc)
    return {"samples": int(k), "qf_max": float(ef.max()), "qf_median": float(np.median(ef)),
            "qc_max": float(ec.max()), "qc_median": float(np.median(ec)),
            "same_cycles": int(np.all(form["cycles"][:k] == ocyc, axis=1).sum())}


# ------------------------------------------------ driver-visible workloads
# Bounded versions of the report workloads (cfg1..cfg5), run by the default
# benchmark after the headline so that every configuration is measured in the
# same run. Each entry states what was reduced relative to the full workload.

def _kl_write_bytes(n):
    """Coefficient bytes the KL pass writes per sample in an FP32+IR solve whose finest grid
    is n: the FP64 field on the two top grids, the FP32 field on every grid down to 4^2."""
    grids = [n >> k for k in range((n // 4).bit_length())]
    return 8 * (grids[0] ** 2 + grids[1] ** 2) + 4 * sum(g * g for g in grids)


def _kl_mfma(prof, dtype, samples=0, n=0):
    ms, launches, flops = prof["kl"]
    if not launches or ms <= 0:
        return None
    peak = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}[dtype]
    tf = flops / (ms * 1e-3) / 1e12
    out = {"tflops": round(tf, 2), "peak_tflops": peak, "frac": round(tf / peak, 4), "ms": round(ms, 3)}
    if samples and n:
        gbs = _kl_write_bytes(n) * samples / (ms * 1e-3) / 1e9
        out.update(write_gbs=round(gbs, 1), hbm_frac=round(gbs / 8000.0, 4),
                   ms_at_hbm_peak=round(_kl_write_bytes(n) * samples / 8e12 * 1e3, 3))
    return out


def _fill_gbs(torch, nbytes, reps=3):
    """Rate of a plain device fill of nbytes (a store-only reference for the KL writes)."""
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    buf.fill_(0.0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        buf.fill_(1.0)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del buf
    return round(nbytes / (ms * 1e-3) / 1e9, 1)


def compact_reports(torch, fmgmc, inputs, args):
    from oracle import oracle as O
    out = {}
    t_all = time.perf_counter()
    # d1: cfg1 in full, FP64, every sample against the oracle
    cfg = dict(sigma2=1.0, corr_len=0.3, n_modes=64, n_levels=3, n0=16)
    ns = [1000, 1000, 1000]
    xis = [inputs.mc_normals(n, cfg["n_modes"], config=1, level=l) for l, n in enumerate(ns)]
    xd = [_dev(torch, x) for x in xis]
    res = [_bufs(torch, n) for n in ns]
    with fmgmc.Context(**cfg, solver="fp64") as ctx:
        ctx.solve_levels(xd, [o[0] for o in res], [o[1] for o in res])
        t0 = _t(torch)
        rc = ctx.solve_levels(xd, *[[o[k] for o in res] for k in range(4)])
        dt = _t(torch) - t0
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    ef, ec, same = [], [], 0
    for l in range(3):
        of, oc, ocy, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, cfg["n0"] << l, l, xis[l],
                                       nthreads=O.max_threads())
        ef.append(np.abs(res[l][0].cpu().numpy() - of) / np.abs(of))
        if l:
            ec.append(np.abs(res[l][1].cpu().numpy() - oc) / np.abs(oc))
        same += int(np.all(res[l][2].cpu().numpy() == ocy, axis=1).sum())
    est = fmgmc.estimate([o[0] for o in res], [o[1] for o in res])
    out["d1_cfg1"] = {"samples_per_s": round(sum(ns) / dt, 1), "status": int(rc),
                      "qf_max_rel_err_vs_oracle": float(np.concatenate(ef).max()),
                      "qc_max_rel_err_vs_oracle": float(np.concatenate(ec).max()),
                      "same_cycles_as_oracle": f"{same}/{sum(ns)}", "estimate": est["mean"],
                      "workload": "3 levels 16^2/32^2/64^2, 1000 samples each, FP64, rel-res 1e-10 (full size)"}
    log("reports: d1 done")
    # d2: cfg2 with the frozen N_l scaled by 1/report_div, both forms
    cfg = dict(CFG)
    div = args.report_div
    ns = [max(16, n // div) for n in _cfg2_counts()]
    xd = [_dev(torch, inputs.mc_normals_blocked(0, n, cfg["n_modes"], config=2, level=l)) for l, n in enumerate(ns)]
    d2 = {"n_l": ns, "workload": f"5 levels 32^2..512^2, the frozen N_l divided by {div}, rel-res 1e-10"}
    Q = {}
    for f in ("fp32_ir", "fp64"):
        res = [_bufs(torch, n) for n in ns]
        with fmgmc.Context(**cfg, solver=f, max_batch=2048, max_cycles=60, w_max_n=args.wmax,
                           **(dict(inner_first=args.inner_first) if f == "fp32_ir" else {})) as ctx:
            ctx.solve_levels(xd, [o[0] for o in res], [o[1] for o in res])
            t0 = _t(torch)
            rc = ctx.solve_levels(xd, *[[o[k] for o in res] for k in range(4)])
            dt = _t(torch) - t0
        est = fmgmc.estimate([o[0] for o in res], [o[1] for o in res])
        Q[f] = [(o[0].cpu().numpy(), o[1].cpu().numpy()) for o in res]
        d2[f] = {"samples_per_s": round(sum(ns) / dt, 1), "status": int(rc), "estimate": est["mean"],
                 "var_of_mean": est["var_of_mean"], "sampling_rmse": float(np.sqrt(est["var_of_mean"])),
                 "flagged": int(sum(int((o[3] != 0).sum().item()) for o in res))}
    err = {f: [] for f in Q}
    for l in range(len(ns)):
        k = min(8, ns[l])
        xo = xd[l][:k].cpu().numpy()
        of, oc = _oracle_subset(cfg, l, xo, 1e-12)
        for f in Q:
            err[f].append(np.abs(Q[f][l][0][:k] - of) / np.abs(of))
            if l:
                err[f].append(np.abs(Q[f][l][1][:k] - oc) / np.abs(oc))
    for f in Q:
        e = np.concatenate(err[f])
        d2[f]["qoi_rel_err_vs_oracle_at_1e-12"] = {"max": float(e.max()), "median": float(np.median(e)),
                                                   "values": int(e.size)}
    d2["estimate_rel_diff_fp32_ir_vs_fp64"] = abs(d2["fp32_ir"]["estimate"] - d2["fp64"]["estimate"]) / abs(
        d2["fp64"]["estimate"])
    out["d2_cfg2"] = d2
    del xd
    log("reports: d2 done")
    # d3: cfg3 reduced to 2^m Sobol' points x 16 shifts per level against as many MC samples;
    # KL contraction in FP64 / FP32 / BF16 on the Sobol' points, with its matrix-core rate
    cfg = dict(sigma2=2.0, corr_len=0.1, n_modes=512, n_levels=4, n0=64)
    m_log2, R = args.report_qmc_log2, 16
    Np = R << m_log2
    d3 = {"workload": f"4 levels 64^2..512^2, 2^{m_log2} Sobol' points x {R} digital shifts per level against "
                      f"{Np} i.i.d. samples per level (equal cost), FP32+IR to 1e-10", "levels": []}
    tot = {"var_rqmc": 0.0, "var_mc": 0.0}
    prec = {"kl_fp64": "fp64", "kl_fp32": "fp32", "kl_bf16": "bf16"}
    ctxs = {k: fmgmc.Context(**cfg, solver="fp32_ir", kl_prec=p, max_batch=2048, max_cycles=60,
                             w_max_n=args.wmax, inner_first=args.inner_first) for k, p in prec.items()}
    kl_rate = {}
    for l in range(cfg["n_levels"]):
        xq = _dev(torch, inputs.rqmc_normals(cfg["n_modes"], m_log2, R, config=3, level=l))
        row = {"n": cfg["n0"] << l}
        q = {}
        for k, ctx in ctxs.items():
            qf, qc, c, fl = _bufs(torch, Np)
            ctx.profile(l == cfg["n_levels"] - 1)
            ctx.solve_level(l, xq, qf, qc, c, fl)
            ctx.profile(False)
            pr = ctx.profile_read()
            if l == cfg["n_levels"] - 1:
                kl_rate[k] = _kl_mfma(pr, prec[k], Np, cfg["n0"] << l)
            q[k] = torch.cat([qf, qc]).cpu().numpy()
            if k == "kl_fp64":
                e = fmgmc.estimate([qf], [qc], n_shifts=R)
                row["rqmc_var_of_mean"] = e["var_of_mean"]
                tot["var_rqmc"] += e["var_of_mean"]
        for k in ("kl_fp32", "kl_bf16"):
            m = q["kl_fp64"] != 0
            row[f"{k}_qoi_rel_err"] = _rel(q[k][m], q["kl_fp64"][m])
        xm = _dev(torch, inputs.mc_normals_blocked(0, Np, cfg["n_modes"], config=3, level=l))
        qf, qc, c, fl = _bufs(torch, Np)
        ctxs["kl_fp64"].solve_level(l, xm, qf, qc, c, fl)
        e = fmgmc.estimate([qf], [qc])
        row["mc_var_of_mean"] = e["var_of_mean"]
        row["variance_ratio_mc_over_rqmc"] = e["var_of_mean"] / row["rqmc_var_of_mean"]
        tot["var_mc"] += e["var_of_mean"]
        d3["levels"].append(row)
        del xq, xm
    for c in ctxs.values():
        c.close()
    d3["variance_ratio_mc_over_rqmc_total"] = tot["var_mc"] / tot["var_rqmc"]
    n_top = cfg["n0"] << (cfg["n_levels"] - 1)
    d3["kl_contraction_at_512"] = {
        "note": "KL synthesis rate on the 512^2 level (FP64: the separable factorisation; FP32 / BF16: the dense "
                "samples x 512 modes x cells contraction with FP32 accumulation), flops of the path taken over "
                "the kernel's event-timed duration, against the dense matrix-core peak of its input type; "
                "write_gbs: the coefficient pyramid it writes over the same duration, against 8 TB/s "
                "(ms_at_hbm_peak: the bound those writes set); plain_fill_gbs: a store-only device fill of "
                "one launch's bytes",
        "bytes_written_per_sample": _kl_write_bytes(n_top),
        "plain_fill_gbs": _fill_gbs(torch, _kl_write_bytes(n_top) * 2048),
        **{k: v for k, v in kl_rate.items()}}
    out["d3_cfg3"] = d3
    log("reports: d3 done")
    # d4: cfg4 in full, all levels in one call
    cfg = dict(sigma2=3.0, corr_len=0.05, n_modes=1024, n_levels=6, n0=32)
    ns = [42451, 15007, 5306, 1875, 663, 234]
    xd = [_dev(torch, inputs.mc_normals_blocked(0, n, cfg["n_modes"], config=4, level=l)) for l, n in enumerate(ns)]
    res = [_bufs(torch, n) for n in ns]
    with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=512, max_cycles=60) as ctx:
        ctx.solve_levels(xd, [o[0] for o in res], [o[1] for o in res])
        t0 = _t(torch)
        rc = ctx.solve_levels(xd, *[[o[k] for o in res] for k in range(4)])
        dt = _t(torch) - t0
    k = 4
    of, oc = _oracle_subset(cfg, 5, xd[5][:k].cpu().numpy(), 1e-10)
    est = fmgmc.estimate([o[0] for o in res], [o[1] for o in res])
    out["d4_cfg4"] = {"samples_per_s": round(sum(ns) / dt, 1), "status": int(rc),
                      "flagged": int(sum(int((o[3] != 0).sum().item()) for o in res)),
                      "cycles_mean_per_level": [[round(float(x), 3) for x in o[2].double().mean(0).cpu().numpy()]
                                                for o in res],
                      "qf_1024_rel_err_vs_oracle": _rel(res[5][0][:k].cpu().numpy(), of),
                      "qc_1024_rel_err_vs_oracle": _rel(res[5][1][:k].cpu().numpy(), oc),
                      "estimate": est["mean"], "var_of_mean": est["var_of_mean"],
                      "workload": f"6 levels 32^2..1024^2, sigma2=3, corr_len=0.05, 1024 modes, N_l = {ns} "
                                  "(65536, full size), FP32+IR to 1e-10, all levels in one solve_levels call"}
    del xd
    log("reports: d4 done")
    # d5: the committed network on 1024 unseen samples at 512^2 against the plain start
    cfg = dict(CFG)
    xi_te = _dev(torch, inputs.mc_normals(1024, cfg["n_modes"], config=5, level=LEVEL,
                                          purpose=inputs.PURPOSE_CNN_TEST))
    S = xi_te.shape[0]
    outs = {}
    with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=S, max_cycles=60, w_max_n=args.wmax,
                       inner_first=args.inner_first) as ctx, fmgmc.Cnn(path=WEIGHTS) as net:
        for name, cnn, mn, mx in (("plain", None, 256, 0), ("warm_256", net, 256, 256), ("warm_512", net, 512, 0),
                                  ("warm_both", net, 256, 0)):
            ctx.set_warm_start(cnn, min_n=mn, max_n=mx)
            qf, qc, cyc, fl = _bufs(torch, S)
            ctx.solve_level(LEVEL, xi_te, qf, qc, cyc, fl)
            t0 = _t(torch)
            for _ in range(3):
                ctx.solve_level(LEVEL, xi_te, qf, qc, cyc, fl)
            dt = (_t(torch) - t0) / 3
            outs[name] = (qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy(), dt)
    p = outs["plain"]
    ep = fmgmc.estimate([p[0]], [p[1]])["mean"]
    d5 = {"cycles_plain": [round(float(x), 4) for x in p[2].mean(0)], "samples_per_s_plain": round(S / p[4], 1),
          "workload": "1024 unseen samples (test stream) at 512^2 / 256^2 of the 5-level config, the committed "
                      "network on the 256^2 stage only (warm_256), the 512^2 stage only (warm_512) or both "
                      "(warm_both), FP32+IR to 1e-10"}
    for name in ("warm_256", "warm_512", "warm_both"):
        w = outs[name]
        ew = fmgmc.estimate([w[0]], [w[1]])["mean"]
        d5[name] = {"cycles_warm": [round(float(x), 4) for x in w[2].mean(0)],
                    "cycles_saved": [round(float(x), 4) for x in p[2].mean(0) - w[2].mean(0)],
                    "warm_rejected": int(((w[3] & fmgmc.FLAG_WARM_REJECTED) != 0).sum()),
                    "samples_per_s_warm": round(S / w[4], 1), "estimate_rel_diff": abs(ew - ep) / abs(ep)}
    out["d5_cfg5"] = d5
    log("reports: d5 done")
    out["seconds"] = round(time.perf_counter() - t_all, 1)
    return out


# ----------------------------------------------------------------- reports
# Each report workload runs one configuration end to end on the GPU and
# prints one JSON line: correctness against the oracle on a subset, the
# estimator, and throughput. They are not the headline measurement.

def _t(torch):
    torch.cuda.synchronize()
    return time.perf_counter()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _bufs(torch, S):
    return (torch.zeros(S, dtype=torch.float64, device="cuda"), torch.zeros(S, dtype=torch.float64, device="cuda"),
            torch.zeros((S, 2), dtype=torch.int32, device="cuda"), torch.zeros(S, dtype=torch.uint8, device="cuda"))


def _rel(a, b):
    r = np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)
    return dict(max=float(r.max()), median=float(np.median(r))) if r.size else None


def _oracle_subset(cfg, level, xi, tol):
    from oracle import oracle as O
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    qf, qc, cyc, fl = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, cfg["n0"] << level, level, xi, tol=tol,
                                    nthreads=O.max_threads())
    return qf, qc


def report_cfg1(torch, fmgmc, inputs, args):
    """3 levels (16^2, 32^2, 64^2), 1000 samples each, FP64, every sample against the oracle."""
    from oracle import oracle as O
    cfg = dict(sigma2=1.0, corr_len=0.3, n_modes=64, n_levels=3, n0=16)
    ns = [1000, 1000, 1000]
    xis = [inputs.mc_normals(n, cfg["n_modes"], config=1, level=l) for l, n in enumerate(ns)]
    xd = [_dev(torch, x) for x in xis]
    out = [_bufs(torch, n) for n in ns]
    with fmgmc.Context(**cfg, solver="fp64") as ctx:
        ctx.solve_levels(xd, [o[0] for o in out], [o[1] for o in out])
        t0 = _t(torch)
        for _ in range(args.steps):
            rc = ctx.solve_levels(xd, [o[0] for o in out], [o[1] for o in out], [o[2] for o in out],
                                  [o[3] for o in out])
        dt = (_t(torch) - t0) / args.steps
    est = fmgmc.estimate([o[0] for o in out], [o[1] for o in out])
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    lv, oq = [], []
    for l in range(3):
        of, oc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, cfg["n0"] << l, l, xis[l],
                                        nthreads=O.max_threads())
        oq.append((of, oc))
        g = out[l][0].cpu().numpy()
        gc = out[l][1].cpu().numpy()
        same = np.all(out[l][2].cpu().numpy() == ocyc, axis=1)
        lv.append(dict(n=cfg["n0"] << l, samples=ns[l], qf_rel_err=_rel(g, of),
                       qc_rel_err=_rel(gc[oc != 0], oc[oc != 0]) if l else None,
                       same_cycle_counts=float(same.mean()), flags=int(out[l][3].cpu().numpy().sum())))
    ost = [O.level_stats(of, oc) for of, oc in oq]
    omean = sum(s["mean_y"] for s in ost)
    return {"metric": "cfg1 FP64 FMG-MLMC, all samples against the oracle", "value": round(sum(ns) / dt, 1),
            "unit": "samples/s", "status": int(rc), "levels": lv, "estimate": est["mean"], "oracle_estimate": omean,
            "estimate_rel_diff": abs(est["mean"] - omean) / abs(omean), "var_of_mean": est["var_of_mean"],
            "config": {"workload": "3 levels 16^2/32^2/64^2, sigma2=1, corr_len=0.3, 64 KL modes, 1000 samples "
                                   "per level, FP64 FMG to rel-res 1e-10, all levels in one solve_levels call"}}


def _cfg2_counts():
    with open(os.path.join(ROOT, "tests", "golden", "cfg2_nl.json")) as f:
        return json.load(f)["n_l"]


def report_cfg2(torch, fmgmc, inputs, args):
    """The 5-level estimate with the frozen per-level counts, FP64 and FP32+IR."""
    cfg = dict(CFG)
    ns = _cfg2_counts()
    L = len(ns)
    R = max(1, -(-ns[0] // (1 << 21)))  # rounds of at most 2M level-0 samples
    Q = {f: [[np.empty(n), np.empty(n)] for n in ns] for f in ("fp64", "fp32_ir")}
    cyc = {f: [np.empty((n, 2), np.int32) for n in ns] for f in Q}
    tsolve = {f: 0.0 for f in Q}
    tseq = 0.0
    flags = {f: 0 for f in Q}
    ctxs = {f: fmgmc.Context(**cfg, solver=f, max_batch=2048, max_cycles=60) for f in Q}
    for r in range(R):
        lo = [n * r // R for n in ns]
        hi = [n * (r + 1) // R for n in ns]
        xd = [_dev(torch, inputs.mc_normals_blocked(lo[l], hi[l] - lo[l], cfg["n_modes"], config=2, level=l))
              for l in range(L)]
        for f, ctx in ctxs.items():
            out = [_bufs(torch, hi[l] - lo[l]) for l in range(L)]
            if r == 0:  # untimed warm-up (workspaces, code objects)
                ctx.solve_levels(xd, [o[0] for o in out], [o[1] for o in out])
            t0 = _t(torch)
            ctx.solve_levels(xd, [o[0] for o in out], [o[1] for o in out], [o[2] for o in out], [o[3] for o in out])
            tsolve[f] += _t(torch) - t0
            for l in range(L):
                Q[f][l][0][lo[l]:hi[l]] = out[l][0].cpu().numpy()
                Q[f][l][1][lo[l]:hi[l]] = out[l][1].cpu().numpy()
                cyc[f][l][lo[l]:hi[l]] = out[l][2].cpu().numpy()
                flags[f] += int((out[l][3].cpu().numpy() != 0).sum())
            if f == "fp32_ir":  # the same round level by level, one after another
                t0 = _t(torch)
                for l in range(L):
                    ctx.solve_level(l, xd[l], out[l][0], out[l][1])
                tseq += _t(torch) - t0
        log(f"cfg2 round {r + 1}/{R} done")
        del xd
    for c in ctxs.values():
        c.close()
    from oracle import oracle as O
    res = {}
    for f in Q:
        est = fmgmc.estimate([q[0] for q in Q[f]], [q[1] for q in Q[f]])
        ost = [O.level_stats(q[0], q[1]) for q in Q[f]]
        res[f] = dict(samples_per_s=round(sum(ns) / tsolve[f], 1), seconds=round(tsolve[f], 3),
                      estimate=est["mean"], var_of_mean=est["var_of_mean"],
                      sampling_rmse=float(np.sqrt(est["var_of_mean"])),
                      oracle_stats_of_same_q=sum(s["mean_y"] for s in ost), flagged=flags[f],
                      cycles_mean=[[round(float(c[:, 0].mean()), 3), round(float(c[:, 1].mean()), 3)]
                                   for c in cyc[f]],
                      var_y=[float(s["var_y"]) for s in ost])
    res["fp32_ir"]["sequential_levels_samples_per_s"] = round(sum(ns) / tseq, 1)
    # per-sample QoI error against the oracle driven to 1e-12 (first 16 samples per level)
    err = {f: [] for f in Q}
    for l in range(L):
        k = min(16, ns[l])
        xi = inputs.mc_normals_blocked(0, k, cfg["n_modes"], config=2, level=l)
        of, oc = _oracle_subset(cfg, l, xi, 1e-12)
        for f in Q:
            e = [np.abs(Q[f][l][0][:k] - of) / np.abs(of)]
            if l:
                e.append(np.abs(Q[f][l][1][:k] - oc) / np.abs(oc))
            err[f].append(np.concatenate(e))
    for f in Q:
        e = np.concatenate(err[f])
        res[f]["qoi_rel_err_vs_oracle_1e-12"] = dict(max=float(e.max()), median=float(np.median(e)),
                                                     samples=int(e.size))
    res["estimate_rel_diff_fp32_ir_vs_fp64"] = abs(res["fp32_ir"]["estimate"] - res["fp64"]["estimate"]) / abs(
        res["fp64"]["estimate"])
    return {"metric": "cfg2 5-level FMG-MLMC estimate", "value": res["fp32_ir"]["samples_per_s"],
            "unit": "samples/s", "n_l": ns, "forms": res,
            "config": {"workload": "5 levels 32^2..512^2, sigma2=1, corr_len=0.2, 256 KL modes, frozen N_l "
                                   "(pilot + optimal allocation for RMSE 1e-3, scaled to 4096 on 512^2), "
                                   "rel-res 1e-10, all levels per solve_levels call, blocked PCG64 inputs"}}


def report_cfg3(torch, fmgmc, inputs, args):
    """RQMC (Sobol' 2^14 x 16 digital shifts; the embedded lattice sequence's first 2^14 points x 16
    random shifts) against MC (2^18 i.i.d.) per level; KL in FP64 / FP32 / BF16 on the Sobol' points."""
    cfg = dict(sigma2=2.0, corr_len=0.1, n_modes=512, n_levels=4, n0=64)
    m_log2, R = 14, 16
    N = R << m_log2
    forms = {"kl_fp64": "fp64", "kl_fp32": "fp32", "kl_bf16": "bf16"}
    ctxs = {k: fmgmc.Context(**cfg, solver="fp32_ir", kl_prec=p, max_batch=2048, max_cycles=60)
            for k, p in forms.items()}
    lv = []
    tot = dict(var_rqmc=0.0, var_lattice=0.0, var_mc=0.0, est_rqmc=0.0, est_lattice=0.0, est_mc=0.0, seconds=0.0)
    kl_est = {k: 0.0 for k in forms}
    for l in range(cfg["n_levels"]):
        xq_host = inputs.rqmc_normals(cfg["n_modes"], m_log2, R, config=3, level=l)
        xq = _dev(torch, xq_host)
        row = dict(n=cfg["n0"] << l)
        q = {}
        for k, ctx in ctxs.items():
            qf, qc, c, fl = _bufs(torch, N)
            t0 = _t(torch)
            ctx.solve_level(l, xq, qf, qc, c, fl)
            dt = _t(torch) - t0
            q[k] = (qf, qc)
            e = fmgmc.estimate([qf], [qc], n_shifts=R)
            kl_est[k] += e["mean"]
            if k == "kl_fp64":
                row.update(rqmc_mean=e["mean"], rqmc_var_of_mean=e["var_of_mean"], seconds=dt,
                           cycles_mean=[round(float(x), 3) for x in c.double().mean(0).cpu().numpy()],
                           flagged=int((fl != 0).sum().item()))
                tot["est_rqmc"] += e["mean"]
                tot["var_rqmc"] += e["var_of_mean"]
                tot["seconds"] += dt
        for k in ("kl_fp32", "kl_bf16"):
            a = torch.cat(q[k]).cpu().numpy()
            b = torch.cat(q["kl_fp64"]).cpu().numpy()
            m = b != 0
            row[f"{k}_qoi_rel_err"] = _rel(a[m], b[m])
        del xq, q
        xl = _dev(torch, inputs.lattice_normals_range(cfg["n_modes"], -1, m_log2, R, config=3, level=l).reshape(N, -1))
        qf, qc, c, fl = _bufs(torch, N)
        ctxs["kl_fp64"].solve_level(l, xl, qf, qc, c, fl)
        e = fmgmc.estimate([qf], [qc], n_shifts=R)
        row.update(lattice_mean=e["mean"], lattice_var_of_mean=e["var_of_mean"],
                   variance_ratio_lattice_over_sobol=e["var_of_mean"] / row["rqmc_var_of_mean"])
        tot["est_lattice"] += e["mean"]
        tot["var_lattice"] += e["var_of_mean"]
        del xl
        xm = _dev(torch, inputs.mc_normals_blocked(0, N, cfg["n_modes"], config=3, level=l))
        qf, qc, c, fl = _bufs(torch, N)
        ctxs["kl_fp64"].solve_level(l, xm, qf, qc, c, fl)
        e = fmgmc.estimate([qf], [qc])
        row.update(mc_mean=e["mean"], mc_var_of_mean=e["var_of_mean"],
                   variance_ratio_mc_over_rqmc=e["var_of_mean"] / row["rqmc_var_of_mean"])
        tot["est_mc"] += e["mean"]
        tot["var_mc"] += e["var_of_mean"]
        # oracle check of the FP64-KL path on the first 4 RQMC points
        xo = np.ascontiguousarray(xq_host[:4])
        del xq_host
        of, oc = _oracle_subset(cfg, l, xo, 1e-12)
        qf4, qc4, _, _ = _bufs(torch, 4)
        ctxs["kl_fp64"].solve_level(l, _dev(torch, xo), qf4, qc4)
        row["fp64_kl_qoi_rel_err_vs_oracle_1e-12"] = _rel(qf4.cpu().numpy(), of)
        lv.append(row)
        log(f"cfg3 level {l} done")
        del xm
    for c in ctxs.values():
        c.close()
    return {"metric": "cfg3 MLQMC vs MLMC estimator variance at equal cost", "value":
            round(tot["var_mc"] / tot["var_rqmc"], 3), "unit": "variance ratio MC/RQMC (total)",
            "variance_ratio_mc_over_lattice": round(tot["var_mc"] / tot["var_lattice"], 3), "levels": lv, "total": tot, "kl_precision_estimates": kl_est,
            "config": {"workload": "4 levels 64^2..512^2, sigma2=2, corr_len=0.1, 512 KL modes, 2^14 Sobol' "
                                   "points x 16 digital shifts and 2^14 lattice points x 16 random shifts per level vs 2^18 i.i.d.; FP32+IR to 1e-10; "
                                   "KL contraction in FP64, FP32 and BF16"}}


def report_cfg4(torch, fmgmc, inputs, args):
    """6 levels 32^2..1024^2 at once (65536 samples), FP32+IR: sequential vs concurrent vs autotuned."""
    cfg = dict(sigma2=3.0, corr_len=0.05, n_modes=1024, n_levels=6, n0=32)
    ns = [42451, 15007, 5306, 1875, 663, 234]
    L = len(ns)
    xd = [_dev(torch, inputs.mc_normals_blocked(0, n, cfg["n_modes"], config=4, level=l)) for l, n in enumerate(ns)]
    out = [_bufs(torch, n) for n in ns]
    # concurrent levels run on one lane (host thread + stream) per hardware queue
    res = {"hardware_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))}
    with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=512, max_cycles=60) as ctx:
        def seq():
            for l in range(L):
                ctx.solve_level(l, xd[l], out[l][0], out[l][1], out[l][2], out[l][3])

        def conc():
            return ctx.solve_levels(xd, [o[0] for o in out], [o[1] for o in out], [o[2] for o in out],
                                    [o[3] for o in out])
        for name, fn in (("sequential_levels", seq), ("concurrent_levels", conc)):
            fn()
            t0 = _t(torch)
            fn()
            res[name] = round(sum(ns) / (_t(torch) - t0), 1)
            log(f"cfg4 {name}: {res[name]} samples/s")
        ref = [(o[0].cpu().numpy().copy(), o[1].cpu().numpy().copy()) for o in out]
        t0 = time.perf_counter()
        sched = [ctx.autotune(l, xd[l][:2048]) for l in range(L)]
        res["autotune_seconds"] = round(time.perf_counter() - t0, 2)
        conc()
        t0 = _t(torch)
        rc = conc()
        res["concurrent_autotuned"] = round(sum(ns) / (_t(torch) - t0), 1)
        same = all(np.array_equal(o[0].cpu().numpy(), r[0]) and np.array_equal(o[1].cpu().numpy(), r[1])
                   for o, r in zip(out, ref))
    lv = []
    for l in range(L):
        c = out[l][2].cpu().numpy()
        lv.append(dict(n=cfg["n0"] << l, samples=ns[l], schedule=sched[l],
                       cycles_mean=[round(float(x), 3) for x in c.mean(0)], cycles_max=[int(x) for x in c.max(0)],
                       flagged=int((out[l][3].cpu().numpy() != 0).sum())))
    k = 4
    xo = xd[L - 1][:k].cpu().numpy()
    of, oc = _oracle_subset(cfg, L - 1, xo, 1e-10)
    est = fmgmc.estimate([o[0] for o in out], [o[1] for o in out])
    # convergence factor per cycle of the same algorithm on this rough field:
    # the oracle's residual history at both QoI stages of 4 samples at 256^2
    from oracle import oracle as O
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    fac = []
    for x in xd[3][:4].cpu().numpy():
        o = O.fmg_sample(O.field(256, cfg["corr_len"], tab, x), level=3, tol=1e-10, max_cycles=60, history=True)
        for h in o["hist"]:
            h = h[h > 1e-13]
            fac += list(h[1:] / h[:-1])
    vfac = {"max": round(float(max(fac)), 4), "geomean": round(float(np.exp(np.mean(np.log(fac)))), 4),
            "n": 256, "samples": 4}
    return {"metric": "cfg4 uneven-size batched stress", "value": res["concurrent_autotuned"], "unit": "samples/s",
            "status": int(rc), "throughput": res, "autotuned_results_identical": bool(same), "levels": lv,
            "cycle_factor_oracle_256": vfac,
            "estimate": est["mean"], "var_of_mean": est["var_of_mean"],
            "qf_1024_rel_err_vs_oracle": _rel(out[L - 1][0][:k].cpu().numpy(), of),
            "qc_1024_rel_err_vs_oracle": _rel(out[L - 1][1][:k].cpu().numpy(), oc),
            "config": {"workload": "6 levels 32^2..1024^2, sigma2=3, corr_len=0.05, 1024 KL modes, N_l = "
                                   f"{ns} (65536 total), FP32+IR to rel-res 1e-10, batch 512"}}


def report_cfg5(torch, fmgmc, inputs, args):
    """Learned warm start at 256^2 / 512^2: train on the method's own solutions, then
    compare FMG from the network's start with plain FMG on unseen samples."""
    cfg = dict(CFG)
    ntr, bt = args.cnn_train, 8
    xi_tr = _dev(torch, inputs.mc_normals_blocked(0, ntr, cfg["n_modes"], config=5, level=LEVEL,
                                                  purpose=inputs.PURPOSE_CNN_TRAIN))
    xi_te = _dev(torch, inputs.mc_normals(1024, cfg["n_modes"], config=5, level=LEVEL,
                                          purpose=inputs.PURPOSE_CNN_TEST))
    res = {}
    with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=args.batch, max_cycles=60) as ctx, \
            fmgmc.Cnn(seed=5) as net:
        hist = []
        t0 = _t(torch)
        chunk = 1024
        for c0 in range(0, ntr, chunk):
            lr = 1e-3 if c0 < ntr // 2 else 3e-4
            hist.extend(ctx.train_cnn(net, LEVEL, xi_tr[c0:c0 + chunk], batch=bt, lr=lr).tolist())
            log(f"cfg5 trained on {min(c0 + chunk, ntr)}/{ntr} samples, residual loss {np.mean(hist[-16:]):.4f}")
        t_train = _t(torch) - t0
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        net.save(os.path.join(ROOT, "gpurun_out", "cnn_cfg2.bin"))
        S = xi_te.shape[0]
        outs = {}
        for name, cnn in (("plain", None), ("warm", net)):
            ctx.set_warm_start(cnn, min_n=256)
            qf, qc, cyc, fl = _bufs(torch, S)
            ctx.solve_level(LEVEL, xi_te, qf, qc, cyc, fl)
            t0 = _t(torch)
            for _ in range(args.steps):
                ctx.solve_level(LEVEL, xi_te, qf, qc, cyc, fl)
            dt = (_t(torch) - t0) / args.steps
            ctx.profile(True)
            ctx.solve_level(LEVEL, xi_te, qf, qc, cyc, fl)
            ctx.profile(False)
            prof = ctx.profile_read()
            outs[name] = (qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy(), dt, prof)
    p, w = outs["plain"], outs["warm"]
    ep = fmgmc.estimate([p[0]], [p[1]])["mean"]
    ew = fmgmc.estimate([w[0]], [w[1]])["mean"]
    cms, cn, cfl = w[5]["cnn"]
    hist = np.asarray(hist)
    res = {
        "train_samples": ntr, "train_stage_solutions": 2 * ntr, "train_seconds": round(t_train, 2),
        "adam_steps": int(hist.size), "residual_loss_first_last": [float(hist[:32].mean()), float(hist[-32:].mean())],
        "cycles_plain": [round(float(x), 4) for x in p[2].mean(0)],
        "cycles_warm": [round(float(x), 4) for x in w[2].mean(0)],
        "cycles_saved": [round(float(x), 4) for x in p[2].mean(0) - w[2].mean(0)],
        "warm_rejected": int(((w[3] & fmgmc.FLAG_WARM_REJECTED) != 0).sum()), "flagged": int((w[3] & 3).sum()),
        "samples_per_s_plain": round(S / p[4], 1), "samples_per_s_warm": round(S / w[4], 1),
        "cnn_ms_per_solve": round(cms, 3), "cnn_tflops": round(cfl / (cms * 1e-3) / 1e12, 2) if cn else None,
        "estimate_plain": ep, "estimate_warm": ew, "estimate_rel_diff": abs(ew - ep) / abs(ep),
        "max_sample_rel_diff_qf": float(np.max(np.abs(w[0] - p[0]) / np.abs(p[0]))),
        "max_sample_rel_diff_qc": float(np.max(np.abs(w[1] - p[1]) / np.abs(p[1]))),
    }
    return {"metric": "cfg5 learned warm start at 256^2/512^2", "value": res["samples_per_s_warm"],
            "unit": "samples/s", "report": res,
            "config": {"workload": f"level 4 of the 5-level config (512^2, coarse stage 256^2), trained on {ntr} "
                                   "samples (two stage solutions each), 1024 unseen test samples, FP32+IR to 1e-10, "
                                   "warm start on both QoI stages"}}


def report_saving(torch, fmgmc, inputs, args):
    """FMG-MLMC against standard MLMC on each level >= 1 of the 5-level configuration:
    Q^c_l from the FMG pass that yields Q^f_l, or from a separate FMG solve on n_l/2."""
    cfg = dict(CFG)
    S = args.samples
    res = []
    # "tolerance": both QoI stages driven to rel-res 1e-10 (the library's stopping rule);
    # "one_cycle": every FMG stage gets one V-cycle (the paper's reading that FMG stage
    # ends are exact), FP64 only
    for form, rule in (("fp32_ir", "tolerance"), ("fp64", "tolerance"), ("fp64", "one_cycle")):
        for level in range(1, cfg["n_levels"]):
            xi = _dev(torch, inputs.mc_normals(S, cfg["n_modes"], config=2, level=level))
            row = {"form": form, "rule": rule, "n": cfg["n0"] << level}
            q = {}
            for mode in (False, True):
                kw = dict(inner_first=args.inner_first, inner_cycles=args.inner) if form == "fp32_ir" else {}
                cyc_cap = 1 if rule == "one_cycle" else 60
                with fmgmc.Context(**cfg, solver=form, max_batch=S, max_cycles=cyc_cap, w_max_n=args.wmax,
                                   separate_coarse=mode, **kw) as ctx:
                    qf, qc, cyc, fl = _bufs(torch, S)
                    ctx.solve_level(level, xi, qf, qc, cyc, fl)
                    t0 = _t(torch)
                    for _ in range(args.steps):
                        ctx.solve_level(level, xi, qf, qc, cyc, fl)
                    dt = (_t(torch) - t0) / args.steps
                key = "separate" if mode else "fmg_mlmc"
                row[key + "_ms"] = round(1e3 * dt, 3)
                row[key + "_cycles"] = [round(float(x), 3) for x in cyc.double().mean(0).cpu().numpy()]
                row[key + "_flagged"] = int(((fl & 3) != 0).sum().item())
                q[key] = (qf.cpu().numpy(), qc.cpu().numpy())
            row["saving"] = round(1.0 - row["fmg_mlmc_ms"] / row["separate_ms"], 4)
            row["max_rel_diff_qc"] = float(np.max(np.abs(q["separate"][1] - q["fmg_mlmc"][1]) / np.abs(q["fmg_mlmc"][1])))
            res.append(row)
            log(f"saving {form} {rule} n {row['n']}: {row['saving']:.3f}")
    fine = [r for r in res if r["n"] == N and r["form"] == "fp32_ir"]
    return {"metric": "FMG-MLMC saving over standard MLMC (separate coarse solve)",
            "value": fine[0]["saving"], "unit": "fraction of the standard-MLMC level cost (512^2, FP32+IR)",
            "paper_closed_form": 0.2, "levels": res,
            "config": {"workload": f"levels 1..4 of the 5-level config (64^2..512^2), {S} samples per level, "
                                   "rel-res 1e-10, one device batch per level"}}


def report_case1(torch, fmgmc, inputs, args):
    """Case I of Table 1 (Dirichlet on all four sides, the paper's 100/0/10/50 scaled by
    1/100; QoI = u(1/2, 1/2)) on the headline workload: 512^2 level of the 5-level
    config, 4096 samples, rel-res 1e-10; Case II (the headline problem) run beside it on
    the same box, and a sampled check against the oracle."""
    cfg = dict(CFG)
    S = args.samples
    xi_host = inputs.mc_normals(S, cfg["n_modes"], config=2, level=LEVEL)
    xi = _dev(torch, xi_host)
    res = {}
    for case in (1, 2):
        for form in ("fp32_ir", "fp64"):
            kw = dict(inner_first=args.inner_first, inner_cycles=args.inner) if form == "fp32_ir" else {}
            with fmgmc.Context(**cfg, solver=form, max_batch=S, max_cycles=60, w_max_n=args.wmax, case=case,
                               rel_tol=args.tol, **kw) as ctx:
                qf, qc, cyc, fl = _bufs(torch, S)
                ctx.solve_level(LEVEL, xi, qf, qc, cyc, fl)
                t0 = _t(torch)
                for _ in range(args.steps):
                    ctx.solve_level(LEVEL, xi, qf, qc, cyc, fl)
                dt = (_t(torch) - t0) / args.steps
                est = fmgmc.estimate([qf], [qc])["levels"][0]
            key = f"case{case}_{form}"
            res[key] = dict(samples_per_s=round(S / dt, 1), ms_per_step=round(1e3 * dt, 2),
                            cycles_mean=[round(float(x), 3) for x in cyc.double().mean(0).cpu().numpy()],
                            flagged=int(((fl & 3) != 0).sum().item()), mean_qf=float(qf.double().mean().item()),
                            mean_y=est["mean_y"], var_y=est["var_y"])
            if case == 1 and form == "fp64":
                pick = [0, 1000, 4095]
                of, oc, ocyc = _oracle_case1(cfg, xi_host[pick], args.tol, args.wmax)
                res[key]["cycles_gpu_vs_oracle"] = [cyc.cpu().numpy()[pick].tolist(), ocyc.tolist()]
                res[key]["qf_rel_err_vs_oracle"] = _rel(qf.cpu().numpy()[pick], of)
                res[key]["qc_rel_err_vs_oracle"] = _rel(qc.cpu().numpy()[pick], oc)
            log(f"case {case} {form}: {res[key]['samples_per_s']} samples/s")
    return {"metric": "Case I FMG-MLMC level throughput", "value": res["case1_fp32_ir"]["samples_per_s"],
            "unit": "samples/s", "forms": res,
            "config": {"workload": f"Case I (Dirichlet 1/0/0.1/0.5 on W/E/S/N, QoI u(1/2,1/2)) on the 512^2 level "
                                   f"of the 5-level config, sigma2=1, corr_len=0.2, 256 KL modes, {S} samples, "
                                   f"rel-res {args.tol:g}; Case II beside it"}}


def _oracle_case1(cfg, xi, tol, wmax):
    from oracle import oracle as O
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    qf, qc, cyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, N, LEVEL, xi, tol=tol, case=1, wmax=wmax,
                                   nthreads=O.max_threads())
    return qf, qc, cyc


def report_adaptive(torch, fmgmc, inputs, args):
    """The adaptive FMG-MLMC (Algorithms 1 and 3) and MLQMC (Algorithm 2) drivers on the
    library: 7-level hierarchy 8^2 .. 512^2 of the 5-level field (sigma2=1, corr_len=0.2,
    256 modes), FP32+IR at rel-res 1e-10."""
    from paper_1910_04727_amd import drivers
    cfg = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=7, n0=8)
    out = {}
    with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=4096, max_cycles=60, w_max_n=args.wmax,
                       inner_first=args.inner_first, inner_cycles=args.inner) as ctx:
        solve = drivers.library_solver(ctx)
        for name, run in (("fmg_mlmc", lambda e: drivers.mlmc(solve, e, 256, 6, cfg["n_levels"], n_init=256)),
                          ("fmg_mlqmc", lambda e: drivers.mlqmc(solve, e, 256, 6, cfg["n_levels"], m_init=6,
                                                                nshift=16))):
            for eps in (4e-3, 1e-3):
                t0 = time.perf_counter()
                r = run(eps)
                dt = time.perf_counter() - t0
                out[f"{name}_eps{eps:g}"] = dict(
                    seconds=round(dt, 2), L=r.L, N=r.N, mean=r.mean, var_of_mean=r.var_of_mean,
                    rmse_bound=math.sqrt(r.var_of_mean + r.bias ** 2), converged=r.converged,
                    alpha=round(r.alpha, 3), beta=round(r.beta, 3), rounds=len(r.rounds),
                    means=[float(m) for m in r.means], V=[float(v) for v in r.V])
                log(f"adaptive {name} eps {eps:g}: L {r.L} N {r.N} {dt:.1f} s")
    return {"metric": "adaptive FMG-MLMC / FMG-MLQMC drivers", "value": out["fmg_mlmc_eps0.001"]["seconds"],
            "unit": "s to RMSE 1e-3 (FMG-MLMC)", "runs": out,
            "config": {"workload": "levels 8^2..512^2 (7), sigma2=1, corr_len=0.2, 256 KL modes, FP32+IR to "
                                   "rel-res 1e-10; MC: blocked PCG64 streams extended as N_l grows; QMC: Sobol' "
                                   "2^m x 16 shifts doubled per level"}}


def report_kl(torch, fmgmc, inputs, args):
    """KL synthesis on the 512^2 level of the cfg3 field (512 modes) inside FP32+IR solves:
    FP64 (separable factorisation), FP32 and BF16 (dense contraction, FP32 accumulation).
    Per launch: the event-timed kernel duration, its matrix-core rate against the dense
    peak of its input type, and its coefficient writes (the FP64 field on the two top
    grids, the FP32 field on every grid of the pyramid) against HBM bandwidth."""
    cfg = dict(sigma2=2.0, corr_len=0.1, n_modes=512, n_levels=4, n0=64)
    level, S, batch = 3, args.samples, min(args.batch, 2048)
    n = cfg["n0"] << level
    xi = _dev(torch, inputs.mc_normals_blocked(0, S, cfg["n_modes"], config=3, level=level))
    per_sample = _kl_write_bytes(n)
    peak = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
    out, q = {}, {}
    for p in ("fp64", "fp32", "bf16"):
        with fmgmc.Context(**cfg, solver="fp32_ir", kl_prec=p, max_batch=batch, max_cycles=60) as ctx:
            qf, qc, c, fl = _bufs(torch, S)
            for _ in range(args.warmup):
                ctx.solve_level(level, xi, qf, qc, c, fl)
            ctx.profile(True)
            for _ in range(args.steps):
                ctx.solve_level(level, xi, qf, qc, c, fl)
            torch.cuda.synchronize()
            ctx.profile(False)
            ms, launches, flops = ctx.profile_read()["kl"]
            q[p] = qf.cpu().numpy()
        per_launch = ms / launches
        samples = S * args.steps / launches
        gbs = per_sample * samples / (per_launch * 1e-3) / 1e9
        tf = flops / (ms * 1e-3) / 1e12
        out[p] = {"ms_per_launch": round(per_launch, 4), "samples_per_launch": samples,
                  "tflops": round(tf, 2), "mfma_peak_tflops": peak[p], "mfma_frac": round(tf / peak[p], 4),
                  "write_gbs": round(gbs, 1), "hbm_frac": round(gbs / 8000.0, 4),
                  "path": "separable" if p == "fp64" else "dense"}
        if p != "fp64":
            out[p]["qoi_rel_diff_vs_fp64_kl"] = _rel(q[p], q["fp64"])
        log(f"kl {p}: {per_launch:.3f} ms per launch, {tf:.1f} TFLOP/s, {gbs:.0f} GB/s of field writes")
    fill = _fill_gbs(torch, per_sample * batch)
    for p in out:
        out[p]["frac_of_plain_fill"] = round(out[p]["write_gbs"] / fill, 4)
    return {"metric": "KL synthesis rate on the 512^2 level", "value": out["bf16"]["tflops"], "unit": "TFLOP/s (BF16)",
            "precisions": out, "bytes_written_per_sample": per_sample, "plain_fill_gbs": fill,
            "config": {"workload": f"cfg3 field (sigma2=2, corr_len=0.1, 512 modes), 512^2 level, {S} samples in "
                                   f"launches of {batch}, inside FP32+IR solves", "steps": args.steps}}


REPORTS = {"case1": report_case1, "cfg1": report_cfg1, "saving": report_saving, "adaptive": report_adaptive, "cfg2": report_cfg2, "cfg3": report_cfg3, "cfg4": report_cfg4,
           "cfg5": report_cfg5, "kl": report_kl}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="headline", choices=["headline"] + sorted(REPORTS),
                    help="headline (default): the 512^2 samples/s line; others print one report line each")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--inner", type=int, default=1)
    ap.add_argument("--inner-first", type=int, default=4, help="FP32 cycles before the first refinement")
    ap.add_argument("--wmax", type=int, default=32, help="W-cycle coarse corrections on grids n <= wmax")
    ap.add_argument("--nu", default="2,2", help="pre,post smoothing sweeps of the FP32 cycles (1..4)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-fuse", action="store_true",
                    help="FP32 cycles back to back as separate post- and pre-smoothing passes")
    ap.add_argument("--forms", default="fp32_ir,fp64,nn_warm")
    ap.add_argument("--cpu-samples", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cnn-train", type=int, default=16384, help="cfg5: level-4 training samples")
    ap.add_argument("--acc-tol", type=float, default=1e-12,
                    help="tolerance of the accuracy record (every form against the oracle; 0 = skip)")
    ap.add_argument("--acc-steps", type=int, default=4, help="timed steps per form of the accuracy record")
    ap.add_argument("--saving-steps", type=int, default=3,
                    help="timed steps of the standard-MLMC comparator (0 = skip)")
    ap.add_argument("--reports", type=int, default=1,
                    help="1: after the headline, bounded runs of every workload (cfg1..cfg5) in the same line")
    ap.add_argument("--report-div", type=int, default=16, help="cfg2 in the line: frozen N_l divided by this")
    ap.add_argument("--report-qmc-log2", type=int, default=10, help="cfg3 in the line: 2^m Sobol' points per shift")
    ap.add_argument("--warm-min-n", type=int, default=256, help="smallest QoI stage the network starts")
    ap.add_argument("--warm-max-n", type=int, default=256,
                    help="largest QoI stage the network starts (0: no bound); on the 512^2 stage the network "
                         "saves no cycle (the cfg5 report measures both)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only (the method's samples are independent, so the "
              "path would shard by sample ranges; that sharding is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_04727_amd import fmgmc, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload != "headline":
        out = REPORTS[args.workload](torch, fmgmc, inputs, args)
        print(json.dumps(out), flush=True)
        return
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
                   "batch": args.batch, "inner_cycles": args.inner, "inner_first": args.inner_first,
                   "w_max_n": args.wmax, "nu_fp32": args.nu, "fuse_cycles": not args.no_fuse},
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
            "warm_rejected": f["warm_rejected"],
            "roofline": roofline(f, args.steps),
            "passes_512": pass_table(f),
            "kl_tflops": round(kl_flops / (kl_ms * 1e-3) / 1e12, 2) if kl_n else None,
            "kl_ms_per_step": round(kl_ms / args.steps, 3) if kl_n else None,
        }
        cnn_ms, cnn_n, cnn_flops = f["prof"]["cnn"]
        if k == "nn_warm":
            out["forms"][k]["warm_stages_n"] = [args.warm_min_n, args.warm_max_n or N]
        if cnn_n:
            out["forms"][k]["cnn_tflops"] = round(cnn_flops / (cnn_ms * 1e-3) / 1e12, 2)
            out["forms"][k]["cnn_ms_per_step"] = round(cnn_ms / args.steps, 3)
    if "nn_warm" in forms and "fp32_ir" in forms:
        a, b = forms["nn_warm"], forms["fp32_ir"]
        out["forms"]["nn_warm_cycles_saved"] = [round(b["cycles_coarse_mean"] - a["cycles_coarse_mean"], 4),
                                                round(b["cycles_fine_mean"] - a["cycles_fine_mean"], 4)]
        out["forms"]["nn_warm_vs_fp32_ir_max_rel_qf_diff"] = float(np.max(np.abs(a["qf"] - b["qf"]) / np.abs(b["qf"])))
    if "fp32_ir" in forms and "fp64" in forms:
        a, b = forms["fp32_ir"], forms["fp64"]
        out["forms"]["ir_vs_fp64_speedup"] = round(a["samples_per_s"] / b["samples_per_s"], 3)
        out["forms"]["ir_vs_fp64_max_rel_qf_diff"] = float(np.max(np.abs(a["qf"] - b["qf"]) / np.abs(b["qf"])))
    # the paper's only performance statement, as context (not a target)
    out["paper_context"] = {
        "saving_from_qc_reuse": 0.2,
        "statement": "FMG-MLMC saves about 20% of the cost of MLMC asymptotically by taking Q^c_l from the FMG "
                     "pass that yields Q^f_l (Abstract; closed form 1/(1+2^gamma), gamma = 2 in 2-D); "
                     "no hardware, precision or timing is given",
    }
    if args.saving_steps and head == "fp32_ir":
        sep = run_form(torch, fmgmc, xi_dev, "fp32_ir", args, steps=args.saving_steps, warmup=1,
                       separate_coarse=True)
        out["paper_context"]["measured_saving_vs_standard_mlmc"] = {
            "value": round(1.0 - H["ms_per_step"] / sep["ms_per_step"], 4),
            "standard_mlmc_ms_per_step": round(sep["ms_per_step"], 2), "fmg_mlmc_ms_per_step": round(H["ms_per_step"], 2),
            "note": "FP32+IR at rel-res 1e-10 on both QoI stages; standard MLMC solves Q^c with its own FMG pass "
                    "to 256^2 (same injected coefficients)"}
    if not args.no_cpu:
        log(f"cpu baseline: oracle on {args.cpu_samples} samples")
        out["cpu_baseline"], ref10 = cpu_baseline(xi, args.cpu_samples, args.tol, args.wmax)
        for k, f in forms.items():
            out["forms"][k][f"qoi_vs_oracle_at_{args.tol:g}"] = qoi_err(f, ref10)
        if args.acc_tol > 0:
            # the mixed-precision bar at one tolerance: each form and the oracle driven to acc_tol
            log(f"accuracy record: oracle at {args.acc_tol:g} on {args.cpu_samples} samples")
            ref = oracle_ref(xi, args.cpu_samples, args.acc_tol, args.wmax)
            rec = {"tol": args.acc_tol, "reference": f"oracle at rel-res {args.acc_tol:g} on the cpu_baseline samples",
                   "bar": 1e-8, "forms": {}}
            for k in forms:
                f = run_form(torch, fmgmc, xi_dev, k, args, tol=args.acc_tol, steps=args.acc_steps, warmup=1)
                e = qoi_err(f, ref)
                rec["forms"][k] = {"samples_per_s": round(f["samples_per_s"], 2),
                                   "cycles_mean": [round(f["cycles_coarse_mean"], 3), round(f["cycles_fine_mean"], 3)],
                                   "flagged_samples": f["flags"], "qoi_vs_oracle": e,
                                   "meets_bar": bool(max(e["qf_max"], e["qc_max"]) <= 1e-8)}
            if "fp32_ir" in rec["forms"] and "fp64" in rec["forms"]:
                rec["ir_vs_fp64_speedup"] = round(rec["forms"]["fp32_ir"]["samples_per_s"] /
                                                  rec["forms"]["fp64"]["samples_per_s"], 3)
            rec["note"] = ("the headline value is measured at rel-res 1e-10; there the stopping rule itself leaves "
                           "QoI differences up to ~3e-7 between any two solver forms at 512^2 (each stops at a "
                           "different iterate of the same discrete problem), so the 1e-8 bar is shown with both "
                           "sides driven to this tolerance")
            out["accuracy_at_tight_tol"] = rec
    if args.reports:
        out["reports"] = compact_reports(torch, fmgmc, inputs, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
