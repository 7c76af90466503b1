"""The learned warm start end to end against the CPU oracle.

The network changes only where a QoI stage starts: every stage still iterates
until ||b - A p|| <= tol ||b||, and a proposed start that does not lower the
residual is replaced by the plain FMG start. Driven to rel-res 1e-12, the
warm-started FP32+IR form must therefore give the oracle's Q^f and Q^c to 1e-8
(the mixed-precision bar), on every sample whose start was kept and on every
sample whose start was rejected. A rejected start is the plain start bitwise,
so such a sample must also repeat the plain form's Q and cycle counts exactly.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc, inputs

pytestmark = pytest.mark.gpu

CFG2 = dict(sigma2=1.0, corr_len=0.2, n_modes=256, n_levels=5, n0=32)
WEIGHTS = os.path.join(os.path.dirname(fmgmc.HERE), "paper_1910_04727_amd", "weights", "cnn_cfg2.bin")
# the benchmark's FP32+IR schedule
SCHED = dict(solver="fp32_ir", inner_first=4, inner_cycles=1, w_max_n=32, max_cycles=80)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def solve(ctx, level, xi):
    S = xi.shape[0]
    qf = torch.zeros(S, dtype=torch.float64, device="cuda")
    qc = torch.zeros_like(qf)
    cyc = torch.zeros((S, 2), dtype=torch.int32, device="cuda")
    fl = torch.zeros(S, dtype=torch.uint8, device="cuda")
    rc = ctx.solve_level(level, torch.from_numpy(np.ascontiguousarray(xi)).to("cuda"), qf, qc, cyc, fl)
    torch.cuda.synchronize()
    return rc, qf.cpu().numpy(), qc.cpu().numpy(), cyc.cpu().numpy(), fl.cpu().numpy()


def oracle(level, xi, tol=1e-12):
    tab = O.kl_table(CFG2["sigma2"], CFG2["corr_len"], CFG2["n_modes"])
    qf, qc, cyc, fl = O.solve_level(CFG2["sigma2"], CFG2["corr_len"], tab, CFG2["n0"] << level, level, xi,
                                    tol=tol, max_cycles=80, wmax=32, nthreads=O.max_threads())
    assert np.all(fl == 0)
    return qf, qc


def rel(a, b):
    return np.abs(a - b) / np.abs(b)


@pytest.mark.parametrize("level,S", [(2, 12), (3, 8)])
def test_warm_start_matches_oracle_at_1e12(level, S):
    """128^2 (coarse stage 64^2) and 256^2 (coarse stage 128^2), warm start on
    every QoI stage n >= 128; the network from the context options."""
    n = CFG2["n0"] << level
    xi = inputs.mc_normals(S, CFG2["n_modes"], config=2, level=level, purpose=3)
    log(f"nn-warm tol 1e-12 level {level} n {n} S {S}")
    with fmgmc.Context(**CFG2, **SCHED, rel_tol=1e-12, cnn_weights=WEIGHTS, warm_min_n=128) as ctx:
        rc, qf, qc, cyc, fl = solve(ctx, level, xi)
    assert rc == fmgmc.OK and not np.any(fl & 7)
    oqf, oqc = oracle(level, xi)
    ef, ec = rel(qf, oqf), rel(qc, oqc)
    kept = (fl & fmgmc.FLAG_WARM_REJECTED) == 0
    log(f"  qf {ef.max():.2e} qc {ec.max():.2e}; starts kept {kept.sum()}/{S}; cycles {cyc.mean(axis=0)}")
    assert ef.max() <= 1e-8 and ec.max() <= 1e-8


def test_warm_start_benchmark_launch_sampled_against_oracle():
    """The benchmark's launch: 4096 samples at 512^2 in one batch, warm start on
    the 256^2 and 512^2 stages, driven to 1e-12; 12 samples recomputed by the
    oracle, among them every sample whose learned start was rejected (up to 4)."""
    S = 4096
    xi = inputs.mc_normals(S, CFG2["n_modes"], config=2, level=4)
    log(f"nn-warm 512^2 S {S} tol 1e-12")
    with fmgmc.Context(**CFG2, **SCHED, rel_tol=1e-12, max_batch=S) as ctx, fmgmc.Cnn(path=WEIGHTS) as net:
        ctx.set_warm_start(net, min_n=256)
        rc, qf, qc, cyc, fl = solve(ctx, 4, xi)
    assert rc == fmgmc.OK and not np.any(fl & 7)
    rejected = np.flatnonzero(fl & fmgmc.FLAG_WARM_REJECTED)
    log(f"  rejected starts: {len(rejected)} {rejected[:8].tolist()}")
    pick = sorted(set(rejected[:4].tolist()) | {0, 511, 1024, 2047, 2192, 3000, 3583, 4095})
    oqf, oqc = oracle(4, xi[pick])
    ef, ec = rel(qf[pick], oqf), rel(qc[pick], oqc)
    log(f"  {len(pick)} samples: qf {ef.max():.2e} qc {ec.max():.2e}")
    assert ef.max() <= 1e-8 and ec.max() <= 1e-8
    assert np.all(np.isfinite(qf)) and np.all(qf > 0)


def test_rejected_start_is_the_plain_start_bitwise():
    """A network whose outputs are blown up by 1e4 makes every proposal worse than
    the plain start: each one is rejected (flag set), and each sample repeats
    the plain form's Q^f, Q^c and cycle counts bit for bit, and the oracle's to 1e-8."""
    level, S = 3, 8
    xi = inputs.mc_normals(S, CFG2["n_modes"], config=2, level=level, purpose=1)
    with fmgmc.Cnn(path=WEIGHTS) as net:
        th = net.params()
        th[-(32 * 9 + 1):] *= 1e4   # output layer weights and bias
        net.set_params(th)
        with fmgmc.Context(**CFG2, **SCHED, rel_tol=1e-12) as ctx:
            plain = solve(ctx, level, xi)
            ctx.set_warm_start(net, min_n=128)
            warm = solve(ctx, level, xi)
    assert plain[0] == fmgmc.OK and warm[0] == fmgmc.OK
    assert np.all(warm[4] == fmgmc.FLAG_WARM_REJECTED), warm[4]
    assert np.array_equal(warm[1], plain[1]) and np.array_equal(warm[2], plain[2])
    assert np.array_equal(warm[3], plain[3])
    oqf, oqc = oracle(level, xi)
    assert rel(warm[1], oqf).max() <= 1e-8 and rel(warm[2], oqc).max() <= 1e-8
