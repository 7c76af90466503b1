"""Pins of the oracle's FMG-MLMC pass (Section 2.5, Algorithm 3) and failure flags."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_04727_amd import inputs

CFG1 = dict(sigma2=1.0, corr_len=0.3, M=64)


def test_vcycle_factor_below_0p2_cfg1():
    """Residual reduction factor below 0.2 on every cycle of every QoI stage,
    on the 3-level config (16^2, 32^2, 64^2), down to the round-off floor.

    What is pinned here is the oracle's default cycle: V(2,2) red-black Gauss-
    Seidel on the QoI stage whose coarse-grid corrections on grids n <= 64 are
    W-cycles (two coarse cycles each), which on these grids makes every
    correction below the stage a W-cycle. Pure V(2,2) is pinned separately
    below to a weaker bound: it does not reach 0.2 on every cycle."""
    tab = O.kl_table(CFG1["sigma2"], CFG1["corr_len"], CFG1["M"])
    worst = 0.0
    for lev, n in enumerate([16, 32, 64]):
        xi = inputs.mc_normals(60, 64, config=1, level=lev)
        for s in range(xi.shape[0]):
            K = O.field(n, CFG1["corr_len"], tab, xi[s])
            out = O.fmg_sample(K, level=lev, tol=1e-13, max_cycles=60, history=True)
            assert out["flags"] == 0
            for h in out["hist"]:
                h = h[h > 1e-13]
                if len(h) > 1:
                    worst = max(worst, float(np.max(h[1:] / h[:-1])))
    assert 0.0 < worst < 0.2, worst


def test_pure_v_cycle_factor_cfg1():
    """Pure V(2,2) (wmax = 0) on the same samples: 90% of the cycles reduce the
    residual by a factor below 0.2 and every cycle by one below 0.3 (measured:
    97% below 0.2, median 0.10, worst 0.25)."""
    tab = O.kl_table(CFG1["sigma2"], CFG1["corr_len"], CFG1["M"])
    fac = []
    for lev, n in enumerate([16, 32, 64]):
        xi = inputs.mc_normals(60, 64, config=1, level=lev)
        for s in range(xi.shape[0]):
            K = O.field(n, CFG1["corr_len"], tab, xi[s])
            out = O.fmg_sample(K, level=lev, tol=1e-13, max_cycles=60, history=True, wmax=0)
            assert out["flags"] == 0
            for h in out["hist"]:
                h = h[h > 1e-13]
                if len(h) > 1:
                    fac.extend((h[1:] / h[:-1]).tolist())
    fac = np.asarray(fac)
    assert np.quantile(fac, 0.9) < 0.2 and fac.max() < 0.3, (np.quantile(fac, 0.9), fac.max())


def test_pure_v_cycle_is_slower_but_converges_to_the_same_q():
    """The W-cycle coarse corrections change the cost, not the converged QoI."""
    tab = O.kl_table(1.0, 0.2, 256)
    xi = inputs.mc_normals(4, 256, config=2, level=2, purpose=1)
    w = O.solve_level(1.0, 0.2, tab, 128, 2, xi, tol=1e-14, max_cycles=100)
    v = O.solve_level(1.0, 0.2, tab, 128, 2, xi, tol=1e-14, max_cycles=100, wmax=0)
    assert np.all(v[2][:, 1] >= w[2][:, 1])
    assert np.max(np.abs(w[0] - v[0]) / np.abs(w[0])) < 1e-11
    assert np.max(np.abs(w[1] - v[1]) / np.abs(w[1])) < 1e-11


def test_hard_sample_converges():
    """A 512^2 sample (index 2192 of the 4096-sample set, log k spanning about
    -3.3..4.05) on which V(2,2) cycles with these coarse operators diverge;
    with W-cycle corrections below 128^2 it converges in a few cycles."""
    tab = O.kl_table(1.0, 0.2, 256)
    xi = inputs.mc_normals(4096, 256, config=2, level=4)[2192]
    K = O.field(256, 0.2, tab, xi)
    out = O.fmg_sample(K, level=1, tol=1e-10, max_cycles=30)
    assert out["flags"] == 0 and out["cycles"][1] <= 8
    bad = O.fmg_sample(K, level=1, tol=1e-10, max_cycles=30, wmax=0)
    assert bad["flags"] & 1


def test_coarse_qoi_is_level_below_fine_qoi():
    """Q^c_l(omega) and Q^f_{l-1}(omega) are the same discrete quantity (corner
    sampling + injection), so with shared xi they agree to the solver tolerance."""
    tab = O.kl_table(1.0, 0.2, 256)
    xi = inputs.mc_normals(6, 256, config=2, level=0)
    lo = O.solve_level(1.0, 0.2, tab, 32, 0, xi, tol=1e-14, max_cycles=80)
    hi = O.solve_level(1.0, 0.2, tab, 64, 1, xi, tol=1e-14, max_cycles=80)
    assert np.max(np.abs(hi[1] - lo[0]) / np.abs(lo[0])) < 1e-11


def test_telescoping_on_fixed_sample_set():
    """sum_l mean(Q^f_l - Q^c_l) = mean(Q^f_L) when every level uses the same xi (Eq. (2))."""
    tab = O.kl_table(1.0, 0.3, 64)
    xi = inputs.mc_normals(20, 64, config=1, level=0)
    total = 0.0
    qf_last = None
    for lev, n in enumerate([16, 32, 64]):
        qf, qc, _, fl = O.solve_level(1.0, 0.3, tab, n, lev, xi, tol=1e-14, max_cycles=80)
        assert np.all(fl == 0)
        total += O.level_stats(qf, qc)["mean_y"]
        qf_last = qf
    ref = O.comp_sum(qf_last) / len(qf_last)
    assert abs(total - ref) <= 1e-11 * abs(ref)


def test_level_zero_has_no_coarse_qoi():
    tab = O.kl_table(1.0, 0.3, 64)
    xi = inputs.mc_normals(4, 64, config=1, level=0)
    qf, qc, cyc, fl = O.solve_level(1.0, 0.3, tab, 16, 0, xi)
    assert np.all(qc == 0.0) and np.all(cyc[:, 0] == 0) and np.all(cyc[:, 1] >= 1)


def test_flags_not_converged_and_nonfinite():
    tab = O.kl_table(1.0, 0.3, 64)
    xi = inputs.mc_normals(3, 64, config=1, level=1)
    _, _, cyc, fl = O.solve_level(1.0, 0.3, tab, 32, 1, xi, tol=1e-10, max_cycles=1)
    assert np.all(fl & 1) and np.all(cyc == 1)
    big = xi * 1e3   # exp overflows to inf somewhere in the field
    qf, _, _, fl = O.solve_level(1.0, 0.3, tab, 32, 1, big, tol=1e-10, max_cycles=5)
    assert np.all(fl & 2)


def test_batched_equals_single():
    tab = O.kl_table(1.0, 0.3, 64)
    xi = inputs.mc_normals(5, 64, config=1, level=2)
    qf, qc, cyc, fl = O.solve_level(1.0, 0.3, tab, 64, 2, xi, nthreads=3)
    for s in range(5):
        K = O.field(64, 0.3, tab, xi[s])
        out = O.fmg_sample(K, level=2)
        assert out["qf"] == qf[s] and out["qc"] == qc[s]
        assert list(out["cycles"]) == list(cyc[s])
