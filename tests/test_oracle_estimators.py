"""Pins of the oracle's estimators (Section 2.1 Eqs. (2)-(5), Section 2.3, Section 2.4)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_04727_amd import inputs


def test_compensated_sum_is_exactly_rounded_on_hard_input():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(10000) * 1e10, rng.standard_normal(10000),
                        -rng.standard_normal(10000) * 1e10])
    rng.shuffle(v)
    assert abs(O.comp_sum(v) - math.fsum(v)) <= 2 * np.spacing(abs(math.fsum(v)) + 1.0)
    w = np.array([1.0, 1e100, 1.0, -1e100])
    assert O.comp_sum(w) == math.fsum(w) == 2.0


def test_level_stats_known_moments():
    rng = np.random.default_rng(1)
    n = 200000
    qf = 3.0 + 2.0 * rng.standard_normal(n)
    qc = 1.0 + 0.5 * rng.standard_normal(n)
    s = O.level_stats(qf, qc)
    y = qf - qc
    assert abs(s["mean_y"] - math.fsum(y) / n) < 1e-14 * abs(s["mean_y"]) + 1e-15
    assert abs(s["var_y"] / np.var(y, ddof=1) - 1) < 1e-12
    assert abs(s["mean_y"] - 2.0) < 5 * math.sqrt(4.25 / n)
    assert abs(s["var_y"] / 4.25 - 1) < 5 * math.sqrt(2.0 / n)
    assert abs(s["var_qf"] / 4.0 - 1) < 5 * math.sqrt(2.0 / n)


def test_rqmc_stats():
    rng = np.random.default_rng(2)
    R, P = 16, 64
    qf = rng.standard_normal(R * P)
    qc = np.zeros(R * P)
    s = O.rqmc_stats(qf, qc, R)
    means = qf.reshape(R, P).mean(axis=1)
    assert np.allclose(s["shift_means"], means, rtol=0, atol=1e-15)
    assert abs(s["mean_y"] - means.mean()) < 1e-15
    assert abs(s["var_mean"] - means.var(ddof=1) / R) < 1e-15


def test_optimal_nl_minimises_cost():
    """The Lagrange-multiplier N_l meets sum V_l/N_l <= eps^2/2 and no feasible
    integer perturbation of one level is cheaper (brute force)."""
    V = np.array([1e-2, 3e-3, 8e-4, 2e-4, 5e-5])
    Cst = np.array([1.0, 4.0, 16.0, 64.0, 256.0])
    eps = 1e-3
    N = O.optimal_nl(V, Cst, eps)
    assert np.sum(V / N) <= eps ** 2 / 2 * (1 + 1e-12)
    # continuous optimum: sum V/N = eps^2/2 exactly before rounding up
    Nc = 2 / eps ** 2 * np.sqrt(V / Cst) * np.sum(np.sqrt(V * Cst))
    assert abs(np.sum(V / Nc) - eps ** 2 / 2) < 1e-18
    cost = np.sum(Nc * Cst)
    rng = np.random.default_rng(3)
    for _ in range(2000):
        f = np.exp(0.3 * rng.standard_normal(len(V)))
        Np = Nc * f
        scale = np.sum(V / Np) / (eps ** 2 / 2)   # rescale onto the constraint
        Np = Np * scale
        assert np.sum(Np * Cst) >= cost * (1 - 1e-12)


def test_inputs_are_reproducible_and_independent_per_level():
    a = inputs.mc_normals(8, 16, config=2, level=3)
    b = inputs.mc_normals(8, 16, config=2, level=3)
    c = inputs.mc_normals(8, 16, config=2, level=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    tail = inputs.mc_normals(5, 16, config=2, level=3, offset=3)
    assert np.array_equal(tail, inputs.mc_normals(8, 16, config=2, level=3)[3:])


def test_blocked_stream_is_position_independent():
    """Any window of the blocked stream equals the same rows of a larger draw;
    blocks are distinct streams; levels and purposes differ."""
    B = inputs.MC_BLOCK
    full = inputs.mc_normals_blocked(B - 3, 10, 4, config=2, level=0, threads=3)
    assert np.array_equal(full[:3], inputs.mc_normals_blocked(B - 3, 3, 4, config=2, level=0))
    assert np.array_equal(full[3:], inputs.mc_normals_blocked(B, 7, 4, config=2, level=0))
    assert not np.array_equal(full[3:5], inputs.mc_normals_blocked(0, 2, 4, config=2, level=0))
    assert not np.array_equal(full, inputs.mc_normals_blocked(B - 3, 10, 4, config=2, level=1))
    z = inputs.mc_normals_blocked(0, 4096, 8, config=2, level=0)
    assert abs(z.mean()) < 4 * (1 / np.sqrt(z.size)) and abs(z.var() - 1) < 0.05


def test_sobol_points_are_a_digital_net():
    """Every 1-D projection of the first 2^k scrambled Sobol' points puts exactly one
    point in each dyadic interval of width 2^-k; an XOR digital shift keeps that."""
    ints = inputs.sobol_ints(32, 10, config=3, level=0)
    for k in [1, 4, 10]:
        top = (ints[: 2 ** k] >> np.uint64(30 - k)).astype(np.int64)
        for d in range(32):
            assert sorted(top[:, d]) == list(range(2 ** k))
    x = inputs.rqmc_normals(8, 6, 4, config=3, level=0)
    assert x.shape == (4 * 64, 8)
    from scipy.special import ndtr
    u = ndtr(x).reshape(4, 64, 8)
    for r in range(4):
        for d in range(8):
            assert sorted(np.floor(u[r, :, d] * 64).astype(int)) == list(range(64))
