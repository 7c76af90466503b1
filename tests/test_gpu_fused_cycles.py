"""FP32 cycles that follow each other with no refinement between them share
one pass over the stage grid: the prolongation and post-smoothing of one cycle
and the pre-smoothing, residual and restriction of the next (the same
half-sweeps, red first, in the same order as the V-cycle of Section 2.5).

Checked through the C ABI on the same seeded inputs:
  - the fused and the separate passes give the same converged QoIs (both
    driven to rel-res 1e-12), and each is within 1e-8 of the FP64 oracle;
  - the fused pass runs exactly where two FP32 cycles join at a marching top
    grid (nu1 + nu2 <= 4), and never otherwise;
  - at 512^2 and rel-res 1e-10 (the bench configuration) the two forms take
    the same cycles on almost every sample and agree to the accuracy of the
    stopping rule.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc, inputs

pytestmark = pytest.mark.gpu

CFG2 = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=5, n0=32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def run(ctx, level, xi):
    S = xi.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros(S, dtype=torch.float64, device="cuda")
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    ctx.profile(True)
    rc = ctx.solve_level(level, torch.from_numpy(np.ascontiguousarray(xi)).cuda(), qf, qc, cyc, fl)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    return rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy(), prof


def oracle(cfg, n, level, xi, **kw):
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    return O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, n, level, xi, **kw)


@pytest.mark.parametrize("nu", [(1, 1), (1, 2), (2, 2), (3, 1), (3, 3)])
def test_fused_matches_separate_and_oracle(nu):
    cfg = CFG2
    level, S = 3, 8
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"fused FP32 cycles nu {nu} n {n} S {S}")
    res = {}
    for fuse in (True, False):
        with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80, nu1=nu[0], nu2=nu[1],
                           w_max_n=32, inner_first=4, fuse_cycles=fuse) as ctx:
            rc, qf, qc, cyc, fl, prof = run(ctx, level, xi)
        assert rc == fmgmc.OK and np.all(fl == 0)
        res[fuse] = (qf, qc, cyc, prof)
    qf1, qc1, cyc1, p1 = res[True]
    qf0, qc0, cyc0, p0 = res[False]
    fusable = nu[0] + nu[1] <= 4
    fuse_ir = fusable and nu[0] <= 2
    # three joins among the four FP32 cycles before the first refinement, on the 256^2 top grid
    assert p1["fused"][1] == (3 if fusable else 0)
    assert p0["fused"][1] == 0 and p0["irpre"][1] == 0
    if fusable and np.array_equal(cyc1, cyc0):
        # each join replaces one post- and one pre-smoothing pass of the top grid
        assert p1["post"][1] == p0["post"][1] - 3
        if fuse_ir:
            # every refinement pass also does the next cycle's pre-smoothing, so no
            # cycle on the top grid has a pre-smoothing pass of its own
            assert p1["pre"][1] == 0 and p1["ir"][1] == 0 and p1["irpre"][1] == p0["ir"][1]
        else:
            assert p1["pre"][1] == p0["pre"][1] - 3 and p1["irpre"][1] == 0
    d = max(np.max(np.abs(qf1 - qf0) / np.abs(qf0)), np.max(np.abs(qc1 - qc0) / np.abs(qc0)))
    oqf, oqc, _, _ = oracle(cfg, n, level, xi, tol=1e-12, max_cycles=80, wmax=32)
    e1 = max(np.max(np.abs(qf1 - oqf) / np.abs(oqf)), np.max(np.abs(qc1 - oqc) / np.abs(oqc)))
    e0 = max(np.max(np.abs(qf0 - oqf) / np.abs(oqf)), np.max(np.abs(qc0 - oqc) / np.abs(oqc)))
    log(f"  fused vs separate {d:.2e}; vs oracle fused {e1:.2e} separate {e0:.2e}; "
        f"cycles fused {cyc1.mean(axis=0)} separate {cyc0.mean(axis=0)}")
    assert d <= 1e-9
    assert e1 <= 1e-8 and e0 <= 1e-8


def test_fused_case1_matches_oracle():
    """Case I (Dirichlet on every side). The fused path's top-stage first refinement
    also forms the start (with the Dirichlet ghost rows) and the correction faces
    (with the north boundary faces): a wrong boundary value there would still
    converge under the refinement, but in more cycles, so the fused and separate
    paths must take the same cycle counts (up to a rounding tie) as well as agree
    on Q."""
    cfg = CFG2
    level, S = 2, 6
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"fused FP32 cycles, Case I, n {n} S {S}")
    out = {}
    for fuse in (True, False):
        with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80, inner_first=4, case=1,
                           fuse_cycles=fuse) as ctx:
            out[fuse] = run(ctx, level, xi)
    rc, qf, qc, cyc, fl, prof = out[True]
    rc0, qf0, qc0, cyc0, fl0, prof0 = out[False]
    assert rc == fmgmc.OK and np.all(fl == 0) and prof["fused"][1] == 3 and prof["irpre"][1] > 0
    assert rc0 == fmgmc.OK and np.all(fl0 == 0)
    assert np.sum(np.any(cyc != cyc0, axis=1)) <= 1 and np.all(np.abs(cyc - cyc0) <= 1)
    d = max(np.max(np.abs(qf - qf0) / np.abs(qf0)), np.max(np.abs(qc - qc0) / np.abs(qc0)))
    oqf, oqc, _, _ = oracle(cfg, n, level, xi, tol=1e-12, max_cycles=80, case=1)
    e = max(np.max(np.abs(qf - oqf) / np.abs(oqf)), np.max(np.abs(qc - oqc) / np.abs(oqc)))
    log(f"  vs oracle {e:.2e}; fused vs separate {d:.2e}; cycles {cyc.mean(axis=0)} / {cyc0.mean(axis=0)}")
    assert d <= 1e-9
    assert e <= 1e-8


def test_fused_512_at_1e10_agrees_with_separate():
    cfg = CFG2
    level, S = 4, 128
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"fused vs separate FP32 cycles at 512^2, rel-res 1e-10, S {S}")
    out = {}
    for fuse in (True, False):
        with fmgmc.Context(**cfg, solver="fp32_ir", max_batch=S, max_cycles=60, w_max_n=32, inner_first=4,
                           fuse_cycles=fuse) as ctx:
            out[fuse] = run(ctx, level, xi)
    (rc1, qf1, qc1, cyc1, fl1, p1), (rc0, qf0, qc0, cyc0, fl0, p0) = out[True], out[False]
    assert rc1 == fmgmc.OK and rc0 == fmgmc.OK and np.all(fl1 == 0) and np.all(fl0 == 0)
    same = np.all(cyc1 == cyc0, axis=1)
    d = np.abs(qf1 - qf0) / np.abs(qf0)
    log(f"  same cycles {same.sum()}/{S}; max rel diff {d.max():.2e}; fused launches {p1['fused'][1]}")
    assert p1["fused"][1] == 3 and p0["fused"][1] == 0
    assert same.mean() >= 0.9
    # both forms stop at rel-res 1e-10, which bounds the QoI error to a few 1e-7 at 512^2
    assert d.max() <= 1e-6
    # every sample of both forms against the oracle at the same tolerance
    oqf, oqc, _, _ = oracle(cfg, 512, level, xi, tol=1e-10, max_cycles=60, wmax=32, nthreads=O.max_threads())
    e1 = max(np.max(np.abs(qf1 - oqf) / np.abs(oqf)), np.max(np.abs(qc1 - oqc) / np.abs(oqc)))
    e0 = max(np.max(np.abs(qf0 - oqf) / np.abs(oqf)), np.max(np.abs(qc0 - oqc) / np.abs(oqc)))
    log(f"  vs oracle (all {S} samples): fused {e1:.2e}, separate {e0:.2e}")
    assert e1 <= 1e-6 and e0 <= 1e-6


def test_fused_at_the_largest_grid():
    """1024^2 top grid (the fused pass then holds 16 ring rows of 1028 cells in LDS), rough
    field of the six-level configuration (sigma2 = 3, corr_len 0.05, 1024 modes)."""
    cfg = dict(sigma2=3.0, corr_len=0.05, n_modes=1024, n_levels=6, n0=32)
    level, S = 5, 4
    xi = inputs.mc_normals(S, cfg["n_modes"], config=4, level=level)
    log(f"fused FP32 cycles at 1024^2, sigma2 3, S {S}, tol 1e-12")
    with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80, w_max_n=32, inner_first=4) as ctx:
        rc, qf, qc, cyc, fl, prof = run(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0) and prof["fused"][1] == 3
    oqf, oqc, _, _ = oracle(cfg, 1024, level, xi, tol=1e-12, max_cycles=80, wmax=32, nthreads=4)
    e = max(np.max(np.abs(qf - oqf) / np.abs(oqf)), np.max(np.abs(qc - oqc) / np.abs(oqc)))
    log(f"  vs oracle {e:.2e}; cycles {cyc.tolist()}")
    assert e <= 1e-8


def test_unconverged_ir_samples_fall_back_to_fp64():
    """FP32 cycles alone cannot take a stage to rel-res 1e-10 (their correction is limited by FP32
    rounding), so with six FP32 cycles before the only refinement and max_cycles = 6 the FP32+IR
    form leaves samples unconverged; each such sample is solved again by the FP64 FMG pass, whose
    outputs it then carries, with FLAG_FP64 set."""
    cfg = CFG2
    level, S = 2, 12
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"FP64 fallback: fp32_ir with inner_first = max_cycles = 6, n 128, S {S}")
    with fmgmc.Context(**cfg, solver="fp32_ir", max_cycles=6, inner_first=6, w_max_n=32) as ctx:
        rc, qf, qc, cyc, fl, _ = run(ctx, level, xi)
    with fmgmc.Context(**cfg, solver="fp64", max_cycles=6, w_max_n=32) as c64:
        rc64, qf64, qc64, cyc64, fl64, _ = run(c64, level, xi)
    fb = (fl & fmgmc.FLAG_FP64) != 0
    log(f"  fell back {fb.sum()}/{S}; rc {rc}; fp64 rc {rc64}")
    assert fb.any()
    assert np.array_equal(qf[fb], qf64[fb]) and np.array_equal(qc[fb], qc64[fb])
    assert np.array_equal(cyc[fb], cyc64[fb]) and np.array_equal(fl[fb] & np.uint8(0xFF ^ fmgmc.FLAG_FP64), fl64[fb])
    assert np.all((fl[~fb] & fmgmc.FLAG_NOTCONV) == 0)
    assert (rc == fmgmc.OK) == (not np.any(fl & fmgmc.FLAG_NOTCONV))
    # a sample the FP64 pass cannot finish either stays flagged, and the call reports it
    with fmgmc.Context(**cfg, solver="fp32_ir", max_cycles=1, w_max_n=32) as ctx:
        rc, qf, qc, cyc, fl, _ = run(ctx, level, xi[:3])
    assert rc == fmgmc.ENOTCONV
    assert np.all(fl & fmgmc.FLAG_NOTCONV) and np.all(fl & fmgmc.FLAG_FP64) and np.all(np.isfinite(qf))
    # non-finite samples are not re-solved
    with fmgmc.Context(**cfg, solver="fp32_ir", w_max_n=32) as ctx:
        rc, qf, qc, cyc, fl, _ = run(ctx, level, xi[:3] * 1e3)
    assert rc == fmgmc.ENONFINITE and np.all(fl & fmgmc.FLAG_NONFINITE) and not np.any(fl & fmgmc.FLAG_FP64)


def test_fall_back_under_all_levels_at_once():
    """The per-level host threads of solve_levels share the FP64 context of the fallback:
    results and flags equal those of one level at a time."""
    cfg = CFG2
    ns = [10, 6]
    xs = [inputs.mc_normals(n, cfg["n_modes"], config=2, level=l, purpose=1) for l, n in enumerate(ns)]
    kw = dict(solver="fp32_ir", max_cycles=6, inner_first=6, w_max_n=32)
    with fmgmc.Context(**cfg, **kw) as ctx:
        one = [run(ctx, l, xs[l])[1:5] for l in range(2)]
    with fmgmc.Context(**cfg, **kw) as ctx:
        xd = [torch.from_numpy(x).cuda() for x in xs]
        qf = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in ns]
        qc = [torch.zeros(n, dtype=torch.float64, device="cuda") for n in ns]
        cy = [torch.zeros((n, 2), dtype=torch.int32, device="cuda") for n in ns]
        fl = [torch.zeros(n, dtype=torch.uint8, device="cuda") for n in ns]
        ctx.solve_levels(xd, qf, qc, cy, fl)
        torch.cuda.synchronize()
    for l in range(2):
        f = fl[l].cpu().numpy()
        log(f"  level {l}: fell back {int(((f & fmgmc.FLAG_FP64) != 0).sum())}/{ns[l]}")
        assert np.any(f & fmgmc.FLAG_FP64)
        assert np.array_equal(qf[l].cpu().numpy(), one[l][0]) and np.array_equal(qc[l].cpu().numpy(), one[l][1])
        assert np.array_equal(cy[l].cpu().numpy(), one[l][2]) and np.array_equal(f, one[l][3])
