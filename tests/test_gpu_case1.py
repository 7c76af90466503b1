"""Case I of Table 1 on the HIP path against the oracle, through the C ABI:
Dirichlet pressure on all four sides (the paper's 100/0/10/50, scaled by
1/100), QoI = u(1/2, 1/2).

Same seeded inputs on both sides; bars as for Case II: FP64 FMG to 1e-10 on
samples with equal cycle counts, FP32 + FP64 refinement to 1e-8 when both
sides iterate to 1e-12. Properties that hold at any size: equal data on every
side give that constant as the QoI of every sample; Q^c_l equals Q^f_{l-1}
on shared inputs; the sample-wise maximum principle.
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
G = fmgmc.BOUNDARY_DEFAULTS[1]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def run_level(ctx, level, xi):
    S = xi.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros(S, dtype=torch.float64, device="cuda")
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    rc = ctx.solve_level(level, torch.from_numpy(np.ascontiguousarray(xi)).cuda(), qf, qc, cyc, fl)
    torch.cuda.synchronize()
    return rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy()


def oracle(cfg, n, level, xi, **kw):
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])
    return O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, n, level, xi, case=1, **kw)


def test_fp64_all_small_levels_chunked():
    """16^2..64^2 (LDS cycles and the first marching grid), ragged count, batches of 16."""
    cfg = CFG1
    with fmgmc.Context(**cfg, max_batch=16, case=1) as ctx:
        for level in range(3):
            n = cfg["n0"] << level
            xi = inputs.mc_normals(37, cfg["n_modes"], config=1, level=level)
            log(f"case I fp64 level {level} n {n} S 37")
            rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
            oqf, oqc, ocyc, ofl = oracle(cfg, n, level, xi)
            assert rc == fmgmc.OK and np.all(fl == 0) and np.all(ofl == 0)
            assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, f"  qf l{level}")
            if level == 0:
                assert np.all(qc == 0)
            else:
                assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, f"  qc l{level}")
            assert np.all((qf > min(G)) & (qf < max(G)))


@pytest.mark.parametrize("level,S", [(2, 9), (3, 5)])
def test_fp64_marching_levels(level, S):
    cfg = CFG2
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"case I fp64 n {n} S {S}")
    with fmgmc.Context(**cfg, case=1) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, _ = oracle(cfg, n, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    assert_same_solution(qf, oqf, cyc[:, 1:], ocyc[:, 1:], 1e-10, "  qf")
    assert_same_solution(qc, oqc, cyc[:, :1], ocyc[:, :1], 1e-10, "  qc")


@pytest.mark.parametrize("level,S", [(0, 24), (2, 8), (3, 4)])
def test_ir_matches_oracle_to_1e8(level, S):
    cfg = CFG2
    n = cfg["n0"] << level
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level, purpose=1)
    log(f"case I fp32+IR tol 1e-12 n {n} S {S}")
    with fmgmc.Context(**cfg, solver="fp32_ir", rel_tol=1e-12, max_cycles=80, case=1) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    oqf, oqc, ocyc, _ = oracle(cfg, n, level, xi, tol=1e-12, max_cycles=80)
    assert rc == fmgmc.OK and np.all(fl == 0)
    ef = np.abs(qf - oqf) / np.abs(oqf)
    log(f"  qf max rel err {ef.max():.2e}; cycles gpu {cyc[:, 1].mean():.1f} oracle {ocyc[:, 1].mean():.1f}")
    assert ef.max() <= 1e-8
    if level > 0:
        assert np.max(np.abs(qc - oqc) / np.abs(oqc)) <= 1e-8


@pytest.mark.parametrize("solver,tol,bound", [("fp64", 1e-10, 1e-10), ("fp32_ir", 1e-12, 1e-8)])
def test_512_batch_sampled_against_oracle(solver, tol, bound):
    cfg = CFG2
    level, S = 4, 128
    xi = inputs.mc_normals(S, cfg["n_modes"], config=2, level=level)
    log(f"case I 512^2 {solver} tol {tol} S {S}")
    with fmgmc.Context(**cfg, solver=solver, rel_tol=tol, max_batch=S, max_cycles=80, case=1) as ctx:
        rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
    assert rc == fmgmc.OK and np.all(fl == 0)
    pick = list(range(0, S, 8)) + [S - 1]
    oqf, oqc, ocyc, _ = oracle(cfg, 512, level, xi[pick], tol=tol, max_cycles=80, nthreads=O.max_threads())
    log(f"  cycles gpu {cyc[pick].tolist()} oracle {ocyc.tolist()}")
    if solver == "fp64":
        assert_same_solution(qf[pick], oqf, cyc[pick][:, 1:], ocyc[:, 1:], bound, "  qf")
        assert_same_solution(qc[pick], oqc, cyc[pick][:, :1], ocyc[:, :1], bound, "  qc")
    else:
        assert np.max(np.abs(qf[pick] - oqf) / np.abs(oqf)) <= bound
        assert np.max(np.abs(qc[pick] - oqc) / np.abs(oqc)) <= bound
    assert np.all((qf > min(G)) & (qf < max(G)))


@pytest.mark.parametrize("solver", ["fp64", "fp32_ir"])
def test_equal_boundary_values_give_that_constant(solver):
    """p = c solves the problem for any field when every side holds c; the FMG
    start reproduces it, so every sample returns c (512^2 included)."""
    cfg = CFG2
    c = 0.37
    # the FP32 form starts a stage from an FP32 solution (c rounded to 1e-8), and a
    # residual of 1e-10 bounds Q only to about that; iterate it to 1e-12
    tol = 1e-10 if solver == "fp64" else 1e-12
    with fmgmc.Context(**cfg, solver=solver, case=1, p_west=c, p_east=c, p_south=c, p_north=c,
                       max_batch=64, rel_tol=tol, max_cycles=80) as ctx:
        for level in (1, 4):
            xi = inputs.mc_normals(64, cfg["n_modes"], config=2, level=level, purpose=1)
            rc, qf, qc, cyc, fl = run_level(ctx, level, xi)
            log(f"  {solver} level {level}: max |Q - c| {np.abs(qf - c).max():.2e}, cycles {cyc[:, 1].max()}")
            assert rc == fmgmc.OK and np.all(fl == 0)
            bound = 1e-12 if solver == "fp64" else 1e-10
            assert np.abs(qf - c).max() <= bound and np.abs(qc - c).max() <= bound


def test_coarse_qoi_equals_the_level_below():
    """Q^c_l (the n_l/2 stage of the level-l pass) and Q^f_{l-1} on shared inputs."""
    cfg = CFG2
    xi = inputs.mc_normals(48, cfg["n_modes"], config=2, level=3, purpose=1)
    with fmgmc.Context(**cfg, case=1, rel_tol=1e-12, max_cycles=80) as ctx:
        _, qf2, _, _, _ = run_level(ctx, 2, xi)
        _, _, qc3, _, _ = run_level(ctx, 3, xi)
    rel = np.abs(qc3 - qf2) / np.abs(qf2)
    log(f"  max |Q^c_3 - Q^f_2| / |Q^f_2| = {rel.max():.2e}")
    assert rel.max() <= 1e-10


def test_cases_differ_and_network_calls_reject_case1():
    cfg = CFG1
    xi = inputs.mc_normals(8, cfg["n_modes"], config=1, level=1)
    with fmgmc.Context(**cfg, solver="fp32_ir", case=1) as c1, fmgmc.Context(**cfg, solver="fp32_ir") as c2:
        _, q1, _, _, _ = run_level(c1, 1, xi)
        _, q2, _, _, _ = run_level(c2, 1, xi)
        assert np.min(np.abs(q1 - q2)) > 1e-3
        net = fmgmc.Cnn(seed=1)
        with pytest.raises(fmgmc.FmgmcError):
            c1.set_warm_start(net, 16)
        net.close()
