"""Full-size and limit cases through the C ABI.

  - The launch configuration the benchmark times (4096 samples at 512^2 in one
    device batch, its FP32 + FP64-refinement schedule), sampled against the
    oracle one sample at a time.
  - The largest grid (1024^2, six levels) against the oracle.
  - A constant field (sigma^2 so small that exp(g) rounds to 1 in every cell)
    at every level up to 1024^2: Case II has the exact solution p = 1 - x
    (in FP64 the FMG start is already exact, since bilinear interpolation
    reproduces linear data), so Q = 1; Case I gives the mean of the four
    boundary values (the symmetry of the square).
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
    qc = torch.zeros_like(qf)
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    rc = ctx.solve_level(level, torch.from_numpy(np.ascontiguousarray(xi)).cuda(), qf, qc, cyc, fl)
    torch.cuda.synchronize()
    return rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy()


def test_benchmark_launch_configuration_sampled_against_oracle():
    cfg = CFG2
    S, level = 4096, 4
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"4096 x 512^2, one batch, FP32+IR schedule (4, 1), W <= 32, tol 1e-12")
    with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_batch=S, max_cycles=80, w_max_n=32,
                       inner_first=4, inner_cycles=1) as ctx:
        rc, qf, qc, cyc, fl = run(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    pick = list(range(0, S, 64)) + [S - 1]  # 65 samples across the batch, both ends included
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    oqf, oqc, _, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, 512, level, xi[pick], tol=1e-12,
                                   max_cycles=80, nthreads=O.max_threads())
    ef = np.abs(qf[pick] - oqf) / np.abs(oqf)
    ec = np.abs(qc[pick] - oqc) / np.abs(oqc)
    log(f"  max rel err qf {ef.max():.2e} qc {ec.max():.2e}; cycles {cyc.mean(0)}")
    assert ef.max() <= 1e-8 and ec.max() <= 1e-8
    assert np.all(np.isfinite(qf)) and np.all(qf > 0) and np.all(qc > 0)


def test_largest_grid_against_oracle():
    cfg = dict(sigma2=3.0, corr_len=0.05, n_modes=1024, n_levels=6, n0=32)
    level = 5
    xi = inputs.mc_normals(4, cfg["n_modes"], config=4, level=level)
    log("1024^2, sigma2 = 3, corr_len 0.05, 1024 modes, FP64, 4 samples")
    with fmgmc.Context(**cfg, rel_tol=1e-10, max_cycles=80) as ctx:
        rc, qf, qc, cyc, fl = run(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    oqf, oqc, ocyc, _ = O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, 1024, level, xi, tol=1e-10,
                                      max_cycles=80, nthreads=4)
    same = np.all(cyc == ocyc, axis=1)
    ef = np.abs(qf - oqf) / np.abs(oqf)
    ec = np.abs(qc - oqc) / np.abs(oqc)
    log(f"  cycles gpu {cyc.tolist()} oracle {ocyc.tolist()}; max rel err qf {ef.max():.2e} qc {ec.max():.2e}")
    assert same.all()
    assert ef.max() <= 1e-10 and ec.max() <= 1e-10


@pytest.mark.parametrize("solver", ["fp64", "fp32_ir"])
def test_constant_field_case2_is_exact_at_every_level(solver):
    cfg = dict(sigma2=1e-300, corr_len=0.2, n_modes=64, n_levels=6, n0=32)
    with fmgmc.Context(**cfg, solver=solver, max_batch=64) as ctx:
        for level in range(6):
            xi = inputs.mc_normals(16, cfg["n_modes"], config=2, level=level)
            rc, qf, qc, cyc, fl = run(ctx, level, xi)
            log(f"  {solver} n {32 << level}: max |Q^f - 1| {np.abs(qf - 1).max():.1e}, cycles {cyc.max(0)}")
            assert rc == fmgmc.OK and np.all(fl == 0)
            # the FP64 pass carries the exact start through; the FP32 form starts a
            # stage from an FP32 solution (1 - x rounded), which the stopping rule
            # (rel-res 1e-10) then bounds only to about that
            bound = 1e-12 if solver == "fp64" else 1e-10
            assert np.abs(qf - 1.0).max() <= bound
            if level > 0:
                assert np.abs(qc - 1.0).max() <= bound


@pytest.mark.parametrize("solver", ["fp64", "fp32_ir"])
def test_constant_field_case1_gives_the_mean_boundary_value(solver):
    cfg = dict(sigma2=1e-300, corr_len=0.2, n_modes=64, n_levels=6, n0=32)
    want = sum(fmgmc.BOUNDARY_DEFAULTS[1]) / 4
    with fmgmc.Context(**cfg, solver=solver, case=1, rel_tol=1e-12, max_cycles=80, max_batch=16) as ctx:
        for level in (0, 3, 5):
            xi = inputs.mc_normals(16, cfg["n_modes"], config=2, level=level)
            rc, qf, qc, cyc, fl = run(ctx, level, xi)
            log(f"  {solver} n {32 << level}: max |Q^f - {want}| {np.abs(qf - want).max():.1e}")
            assert rc == fmgmc.OK and np.all(fl == 0)
            assert np.abs(qf - want).max() <= 1e-10
