"""Parity of the HIP path with the CPU oracle, through the C ABI.

Same seeded inputs on both sides; the oracle runs the same algorithm in plain
FP64. Tolerances:
  - KL field, FP64 contraction: 1e-13 relative per cell (summation order only).
  - FP64 FMG at tol 1e-10: the GPU runs the same cycles as the oracle, so the
    QoIs agree to rounding (1e-10 relative) whenever both stop after the same
    cycle count; rounding can move a sample whose residual sits right at the
    tolerance by one cycle, which changes Q by up to the solver's own error.
  - FP32 cycles + FP64 refinement: QoI within 1e-8 of the oracle when both
    are driven to 1e-12 (the QoI error at rel-res 1e-10 is itself up to ~3e-7
    at 512^2, for any solver form).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc, inputs
from parity_util import assert_same_solution

pytestmark = pytest.mark.gpu

CFG1 = dict(sigma2=1.0, corr_len=0.3, n_modes=64, n_levels=3, n0=16)
CFG2 = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=5, n0=32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to(device="cuda", dtype=dtype)


def run_level(ctx, level, xi):
    S = xi.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros(S, dtype=torch.float64, device="cuda")
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    rc = ctx.solve_level(level, dev(xi), qf, qc, cyc, fl)
    torch.cuda.synchronize()
    return rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy()


def table(cfg):
    return O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])


# ------------------------------------------------------------------ KL field
@pytest.mark.parametrize("level,S,prec", [(0, 70, "fp64"), (1, 33, "fp64"), (3, 70, "fp64"), (1, 9, "fp64_dense"),
                                          (3, 5, "fp64_dense")])
def test_field_fp64_matches_oracle(level, S, prec):
    """FP64: 32^2 (dense contraction, narrow tiles), 64^2 and 256^2 (separable factorisation);
    FP64_DENSE: the dense contraction at 64^2 and 256^2 (row-staged tiles). Ragged sample counts."""
    cfg = CFG2
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"field {prec} level {level} n {n} S {S}")
    with fmgmc.Context(**cfg, kl_prec=prec) as ctx:
        K = torch.zeros((S, n, n), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(level, dev(xi), K)
        torch.cuda.synchronize()
        K = K.cpu().numpy()
    tab = table(cfg)
    worst = 0.0
    for s in range(S):
        ref = O.field(n, cfg["corr_len"], tab, xi[s])
        worst = max(worst, float(np.max(np.abs(K[s] - ref) / ref)))
    log(f"  max rel err {worst:.2e}")
    assert worst <= 1e-13


@pytest.mark.parametrize("prec,bound", [("fp32", 2e-5), ("bf16", 0.25)])
def test_field_reduced_precision_error(prec, bound):
    """FP32 / BF16 contraction with FP32 accumulation: the field error is reported
    (it changes the problem) and bounded by the input rounding of the precision."""
    cfg = dict(sigma2=2.0, corr_len=0.1, n_modes=512, n_levels=1, n0=64)
    S = 40
    xi = inputs.mc_normals(S, 512, config=3, level=0, purpose=1)
    log(f"field {prec} n 64 S {S}")
    with fmgmc.Context(**cfg, kl_prec=prec) as ctx:
        K = torch.zeros((S, 64, 64), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(0, dev(xi), K)
        torch.cuda.synchronize()
        K = K.cpu().numpy()
    tab = table(cfg)
    ref = np.array([O.field(64, cfg["corr_len"], tab, xi[s]) for s in range(S)])
    err = np.abs(np.log(K) - np.log(ref))
    log(f"  {prec}: max |d log K| {err.max():.2e}, rms {np.sqrt((err ** 2).mean()):.2e}")
    assert err.max() <= bound


def _round_bf16(x):
    """float64 -> bfloat16 in one rounding (to nearest, ties to even), as float64: the
    52-bit significand is rounded to 7 bits in place (finite normal inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    one, sh = np.uint64(1), np.uint64(45)
    u = ((u + ((one << np.uint64(44)) - one) + ((u >> sh) & one)) >> sh) << sh
    return u.view(np.float64)


def _kl_operand(cfg, n):
    """B[m][j n + i] = sqrt(lambda_m) phi_{a_m}(i/n) phi_{b_m}(j/n) from the oracle's 1-D pieces."""
    a, b, lam = table(cfg)
    kd = int(max(a.max(), b.max())) + 1
    w, _ = O.kl_1d(cfg["corr_len"], kd)
    x = np.arange(n) / n
    phi = np.array([O.kl_phi(k + 1, w[k], x) for k in range(kd)])
    B = np.sqrt(lam)[:, None, None] * phi[a][:, None, :] * phi[b][:, :, None]
    return B.reshape(len(a), n * n)


@pytest.mark.parametrize("prec,M,n,S", [("bf16", 512, 64, 300), ("fp32", 512, 64, 300), ("bf16", 100, 32, 37),
                                        ("fp32", 100, 32, 37), ("bf16", 64, 16, 5), ("fp32", 48, 16, 5),
                                        ("bf16", 64, 256, 300), ("fp32", 64, 256, 300), ("bf16", 1100, 64, 20),
                                        ("fp32", 600, 64, 20), ("bf16", 4096, 32, 9), ("fp32", 4096, 32, 9)])
def test_field_reduced_precision_rounding(prec, M, n, S):
    """The FP32 / BF16 contraction computes sum_m r(xi_m) r(B_m) with r the rounding of
    each FP64 input to the input type (once, to nearest even), up to FP32
    accumulation: |log K - g| <= M 2^-24 sum_m |r(xi_m) r(B_m)| + 1e-6 (exp and log).
    Ragged sample counts (300 = a full and a partial 256-sample tile, two tiles in one
    workgroup at 256^2), a mode count that is no multiple of 32, grids smaller than one
    64-cell tile, and mode counts beyond what one workgroup keeps in LDS (BF16 > 1024,
    FP32 > 512), up to the largest mode count the library takes (4096)."""
    cfg = dict(sigma2=2.0, corr_len=0.1, n_modes=M, n_levels=1, n0=n)
    xi = inputs.mc_normals(S, M, config=3, level=0, purpose=1)
    log(f"field {prec} M {M} n {n} S {S}")
    with fmgmc.Context(**cfg, kl_prec=prec) as ctx:
        K = torch.zeros((S, n, n), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(0, dev(xi), K)
        torch.cuda.synchronize()
        g = np.log(K.cpu().numpy().reshape(S, n * n))
    B = _kl_operand(cfg, n)
    ref0 = O.field(n, cfg["corr_len"], table(cfg), xi[0]).reshape(-1)
    assert np.max(np.abs(np.exp(xi[0] @ B) / ref0 - 1)) < 1e-12  # the operand above is the oracle's
    if prec == "bf16":
        xr, Br = _round_bf16(xi), _round_bf16(B)
    else:
        xr, Br = xi.astype(np.float32), B.astype(np.float32)
    xr, Br = xr.astype(np.float64), Br.astype(np.float64)
    gref = xr @ Br
    tol = M * 2.0 ** -24 * (np.abs(xr) @ np.abs(Br)) + 1e-6
    err = np.abs(g - gref)
    log(f"  max |log K - g| {err.max():.2e} (max of err/tol {np.max(err / tol):.3f})")
    assert np.all(err <= tol)


@pytest.mark.parametrize("prec,level", [("fp64", 2), ("fp64_dense", 2), ("fp32", 2), ("bf16", 2), ("bf16", 4),
                                        ("fp32", 1)])
def test_field_injection_is_the_coarse_field(prec, level):
    """Cell (I, J) of the grid n/2 is the grid point (2I, 2J) of the grid n (R1, Section 2.5
    coarsening): the field synthesized directly on n/2 equals the fine field at even cells
    bit for bit, for every KL path (the FP32 / BF16 contraction computes each pyramid level
    on its own tiles, so this also holds its coarse levels to the fine values they inject)."""
    cfg = CFG2
    n = cfg["n0"] << level
    S = 37
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"injection {prec} n {n} S {S}")
    with fmgmc.Context(**cfg, kl_prec=prec) as ctx:
        Kf = torch.zeros((S, n, n), dtype=torch.float64, device="cuda")
        Kc = torch.zeros((S, n // 2, n // 2), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(level, dev(xi), Kf)
        ctx.synthesize_field(level - 1, dev(xi), Kc)
        torch.cuda.synchronize()
    Kf, Kc = Kf.cpu().numpy(), Kc.cpu().numpy()
    assert np.array_equal(Kf[:, ::2, ::2], Kc)


def test_solve_reduced_precision_kl():
    """Solves on an FP32 / BF16 field: the fine and coarse QoIs (the coarse one is read
    on the first coarsened coefficient level the KL pass writes) stay within the field's
    rounding of the oracle's, and the cycle counts match."""
    cfg = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=3, n0=32)
    level, S = 2, 40
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=2)
    of, oc, ocy, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), cfg["n0"] << level, level, xi,
                                   nthreads=O.max_threads())
    for solver in ("fp64", "fp32_ir"):
        for prec, bound in (("fp32", 1e-4), ("bf16", 5e-2)):
            with fmgmc.Context(**cfg, kl_prec=prec, solver=solver) as ctx:
                rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
            assert rc == 0 and not fl.any()
            ef, ec = np.max(np.abs(qf / of - 1)), np.max(np.abs(qc / oc - 1))
            same = np.mean(np.all(cyc == ocy, axis=1))
            log(f"  {solver} {prec}: Q^f rel err {ef:.2e}, Q^c rel err {ec:.2e}, same cycles {same:.2f}")
            assert ef <= bound and ec <= bound
            if solver == "fp64" and prec == "fp32":
                assert same >= 0.9


def test_context_mode_table():
    with fmgmc.Context(**CFG2) as ctx:
        a, b, lam = ctx.mode_table()
    oa, ob, olam = table(CFG2)
    assert np.array_equal(a, oa) and np.array_equal(b, ob)
    assert np.max(np.abs(lam / olam - 1)) < 1e-13


# ------------------------------------------------------------------ FP64 FMG
def test_fp64_cfg1_all_levels_chunked():
    """3 levels (16^2, 32^2, 64^2), ragged sample count, batches of 16."""
    cfg = CFG1
    tab = table(cfg)
    with fmgmc.Context(**cfg, max_batch=16) as ctx:
        for level in range(3):
            n = cfg["n0"] << level
            xi = inputs.mc_normals(37, cfg["n_modes"], config=1, level=level)
            log(f"fp64 cfg1 level {level} n {n} S 37")
            rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
            oqf, oqc, ocyc, ofl = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, n, level, xi)
            assert rc == fmgmc.OK and np.all(fl == 0) and np.all(ofl == 0)
            assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, f"  qf l{level}")
            if level == 0:
                assert np.all(qc == 0) and np.all(cyc[:, 0] == 0)
            else:
                assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, f"  qc l{level}")


@pytest.mark.parametrize("level,S", [(2, 9), (3, 5)])
def test_fp64_cfg2_marching_levels(level, S):
    """128^2 and 256^2: the stage and correction smoothing passes run in the
    row-marching kernels; the grids below 64 in LDS."""
    cfg = CFG2
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"fp64 cfg2 level {level} n {n} S {S}")
    with fmgmc.Context(**cfg) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, ofl = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, "  qc")


def test_fp64_nu1_smoothing():
    """V(1,1) cycles: both sides run the same cycle."""
    cfg = CFG2
    level, S = 2, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"fp64 V(1,1) n {n} S {S}")
    with fmgmc.Context(**cfg, nu1=1, nu2=1) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi, nu1=1, nu2=1)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, "  qc")


# ------------------------------------------------------------ FP32 + FP64 IR
@pytest.mark.parametrize("level,S", [(0, 24), (1, 16), (2, 8), (3, 4)])
def test_ir_matches_oracle_to_1e8(level, S):
    """FP32 cycles + FP64 refinement driven to 1e-12 against the oracle: level 0
    (32^2 top grid, cycled in LDS), level 1 (64^2 top grid whose first refinement
    pass forms its start from the 32^2 stage solved in LDS, and writes its
    correction faces), levels 2 and 3."""
    cfg = CFG2
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"fp32+IR tol 1e-12 level {level} n {n} S {S}")
    with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, ofl = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi,
                                        tol=1e-12, max_cycles=80)
    assert rc == fmgmc.OK and np.all(fl == 0)
    ef = np.abs(qf - oqf) / np.abs(oqf)
    log(f"  qf max rel err {ef.max():.2e}; cycles gpu {cyc[:, 1].mean():.1f} oracle {ocyc[:, 1].mean():.1f}")
    assert ef.max() <= 1e-8
    if level > 0:
        ec = np.abs(qc - oqc) / np.abs(oqc)
        log(f"  qc max rel err {ec.max():.2e}")
        assert ec.max() <= 1e-8


def test_ir_at_1e10_error_is_that_of_the_stopping_rule():
    """At rel-res 1e-10 the IR form's QoI error against a converged oracle is of
    the size the FP64 form itself leaves at that tolerance."""
    cfg = CFG2
    level, S = 3, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    with fmgmc.Context(**cfg, solver="fp32_ir") as ctx:
        _, qf, _, _, _ = run_level(ctx, level, xi)
    tab = table(cfg)
    ref, _, _, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, n, level, xi, tol=1e-14, max_cycles=80)
    o10, _, _, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, n, level, xi, tol=1e-10)
    e_ir = np.abs(qf - ref) / np.abs(ref)
    e_64 = np.abs(o10 - ref) / np.abs(ref)
    log(f"rel-res 1e-10 QoI error: IR max {e_ir.max():.2e}, FP64 oracle max {e_64.max():.2e}")
    assert e_ir.max() <= 5 * e_64.max() + 1e-9


# ------------------------------------------------------------------ failures
def test_not_converged_and_nonfinite_flags():
    cfg = CFG1
    xi = inputs.mc_normals(5, 64, config=1, level=1)
    log("flags: max_cycles=1")
    with fmgmc.Context(**cfg, max_cycles=1) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, 1, xi)
    assert rc == fmgmc.ENOTCONV and np.all(fl & fmgmc.FLAG_NOTCONV) and np.all(cyc == 1)
    log("flags: non-finite field")
    with fmgmc.Context(**cfg) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, 1, xi * 1e3)
    assert rc == fmgmc.ENONFINITE and np.all(fl & fmgmc.FLAG_NONFINITE)


def test_empty_batch_and_host_pointers():
    cfg = CFG1
    with fmgmc.Context(**cfg) as ctx:
        z = np.zeros((0, 64))
        e = np.zeros(0)
        assert ctx.solve_level(0, z, e, e.copy()) == fmgmc.OK
        xi = inputs.mc_normals(7, 64, config=1, level=2)
        qf = np.zeros(7)
        qc = np.zeros(7)
        cyc = np.zeros((7, 2), np.int32)
        fl = np.zeros(7, np.uint8)
        log("host-pointer solve")
        assert ctx.solve_level(2, xi, qf, qc, cyc, fl) == fmgmc.OK
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), 64, 2, xi)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  host qf")


# ---------------------------------------------------------------- estimators
def test_estimate_matches_oracle_stats():
    rng = np.random.default_rng(7)
    levels = [(rng.standard_normal(n) + 1.0, 0.3 * rng.standard_normal(n)) for n in (1000, 513, 64)]
    levels[0] = (levels[0][0], np.zeros(1000))
    log("estimate MC")
    out = fmgmc.estimate([dev(a) for a, _ in levels], [dev(b) for _, b in levels])
    tot = 0.0
    var = 0.0
    for l, (a, b) in enumerate(levels):
        s = O.level_stats(a, b)
        g = out["levels"][l]
        for k in ("mean_y", "var_y", "mean_qf", "var_qf", "mean_qc"):
            assert abs(g[k] - s[k]) <= 1e-13 * max(1.0, abs(s[k])), (l, k)
        tot += s["mean_y"]
        var += s["var_y"] / len(a)
    assert abs(out["mean"] - tot) < 1e-13 and abs(out["var_of_mean"] / var - 1) < 1e-12
    log("estimate RQMC")
    qf = rng.standard_normal(16 * 128)
    qc = 0.5 * rng.standard_normal(16 * 128)
    r = fmgmc.estimate([qf], [qc], n_shifts=16)
    s = O.rqmc_stats(qf, qc, 16)
    assert abs(r["levels"][0]["mean_y"] - s["mean_y"]) < 1e-14
    assert abs(r["levels"][0]["var_y"] / s["var_mean"] - 1) < 1e-12


# ------------------------------------------------------- headline size, sampled
@pytest.mark.parametrize("solver,tol,bound", [("fp64", 1e-10, 1e-10), ("fp32_ir", 1e-12, 1e-8)])
def test_512_batch_sampled_against_oracle(solver, tol, bound):
    """512^2 (the finest level of the 5-level config) in a 256-sample batch;
    16 samples spread over the batch recomputed by the oracle."""
    cfg = CFG2
    level, S = 4, 256
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"512^2 {solver} tol {tol} S {S}")
    with fmgmc.Context(**cfg, solver=solver, rel_tol=tol, max_batch=S, max_cycles=80) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    pick = list(range(0, 256, 17)) + [255]
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), 512, level, xi[pick],
                                      tol=tol, max_cycles=80, nthreads=O.max_threads())
    log(f"  cycles gpu {cyc[pick].tolist()} oracle {ocyc.tolist()}")
    if solver == "fp64":
        assert_same_solution(qf[pick], oqf, cyc[pick][:, 1:], ocyc[:, 1:], bound, "  qf")
        assert_same_solution(qc[pick], oqc, cyc[pick][:, :1], ocyc[:, :1], bound, "  qc")
    else:
        assert np.max(np.abs(qf[pick] - oqf) / np.abs(oqf)) <= bound
        assert np.max(np.abs(qc[pick] - oqc) / np.abs(oqc)) <= bound
    # properties that hold for every sample of the batch
    assert np.all(np.isfinite(qf)) and np.all(qf > 0) and np.all(cyc[:, 1] >= 1)


# ------------------------------------------------------------- cycle variants
def test_pure_v_cycles_match_oracle():
    """w_max_n = 0: plain V(2,2) cycles on both sides."""
    cfg = CFG2
    level, S = 2, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=3)
    log(f"fp64 pure V n {n} S {S}")
    with fmgmc.Context(**cfg, w_max_n=0) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi, wmax=0)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, "  qc")


@pytest.mark.parametrize("solver", ["fp64", "fp32_ir"])
def test_hard_high_contrast_sample(solver):
    """Sample 2192 of the 512^2 set (log k from -3.3 to 4.05): pure V-cycles
    diverge on it; the W-cycle coarse corrections converge in a few cycles."""
    cfg = CFG2
    xi = inputs.mc_normals(4096, cfg["n_modes"], config=2, level=4)[2190:2194]
    log(f"hard sample {solver}")
    with fmgmc.Context(**cfg, solver=solver) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, 4, xi)
    assert rc == fmgmc.OK and np.all(fl == 0) and cyc.max() <= 10, cyc
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), 512, 4, xi, nthreads=4)
    if solver == "fp64":
        assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    else:
        assert np.max(np.abs(qf - oqf) / np.abs(oqf)) < 1e-6


@pytest.mark.parametrize("wmax", [32, 16])
def test_fp64_w_threshold_matches_oracle(wmax):
    """W-cycle coarse corrections only on grids n <= wmax, both sides."""
    cfg = CFG2
    level, S = 3, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=3)
    log(f"fp64 wmax {wmax} n {n} S {S}")
    with fmgmc.Context(**cfg, w_max_n=wmax) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi, wmax=wmax)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, "  qc")


@pytest.mark.parametrize("first,inner", [(4, 1), (3, 2)])
def test_ir_cycle_schedule_matches_oracle_to_1e8(first, inner):
    """FP32 cycles before the first FP64 refinement (first) and per refinement
    after it (inner), W-cycles on n <= 32: Q within 1e-8 of the oracle at 1e-12."""
    cfg = CFG2
    level, S = 3, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=3)
    log(f"fp32+IR first {first} inner {inner} wmax 32 n {n} S {S}")
    with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80, w_max_n=32,
                       inner_first=first, inner_cycles=inner) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, _, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi,
                                   tol=1e-12, max_cycles=80, wmax=32)
    assert rc == fmgmc.OK and np.all(fl == 0)
    assert np.all(cyc >= first)
    assert np.all((cyc - first) % inner == 0)
    ef = np.abs(qf - oqf) / np.abs(oqf)
    ec = np.abs(qc - oqc) / np.abs(oqc)
    log(f"  qf {ef.max():.2e} qc {ec.max():.2e}; cycles {cyc.mean(axis=0)}")
    assert ef.max() <= 1e-8 and ec.max() <= 1e-8


def test_field_separable_at_many_modes():
    """1024 modes at correlation length 0.05 (60 1-D modes per axis, the 64-wide
    factorisation) at 128^2 against the oracle."""
    cfg = dict(sigma2=3.0, corr_len=0.05, n_modes=1024, n_levels=6, n0=32)
    level, S = 2, 3
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=4, level=level, purpose=1)
    with fmgmc.Context(**cfg) as ctx:
        K = torch.zeros((S, n, n), dtype=torch.float64, device="cuda")
        ctx.synthesize_field(level, dev(xi), K)
        torch.cuda.synchronize()
        K = K.cpu().numpy()
    tab = table(cfg)
    worst = max(float(np.max(np.abs(K[s] - O.field(n, cfg["corr_len"], tab, xi[s])) /
                         O.field(n, cfg["corr_len"], tab, xi[s]))) for s in range(S))
    log(f"separable 1024 modes n {n}: max rel err {worst:.2e}")
    assert worst <= 1e-12


@pytest.mark.parametrize("solver,bound", [("fp64", 1e-10), ("fp32_ir", 1e-8)])
def test_separate_coarse_solve_is_standard_mlmc(solver, bound):
    """Standard-MLMC comparator: Q^c_l from its own FMG solve on n_l/2, which is
    the oracle's level l-1 solve of the same (injected) field; Q^f_l from a pass
    in which n_l/2 is an intermediate stage, against the oracle's Q^f_l."""
    cfg = CFG2
    level, S = 3, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=3)
    log(f"separate coarse solve, {solver}, n {n}")
    with fmgmc.Context(**cfg, solver=solver, separate_coarse=True, rel_tol=1e-12, max_cycles=80) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    oc, _, ocyc_c, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n // 2, level - 1, xi,
                                     tol=1e-12, max_cycles=80)
    of, _, _, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], table(cfg), n, level, xi, tol=1e-12, max_cycles=80)
    ec = np.abs(qc - oc) / np.abs(oc)
    ef = np.abs(qf - of) / np.abs(of)
    log(f"  qc vs oracle level {level - 1}: {ec.max():.2e} (cycles {cyc[:, 0].mean():.2f} vs {ocyc_c[:, 1].mean():.2f}); "
        f"qf {ef.max():.2e}")
    assert ec.max() <= bound and ef.max() <= 1e-8
