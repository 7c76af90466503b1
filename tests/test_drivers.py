"""Adaptive MLMC / MLQMC drivers (Algorithms 1-3) on solvers with known answers.

A mock level solver returns Y_l = mu_l + sqrt(v_l) xi_0 (xi_0 the first KL
coordinate of each sample, N(0,1)), with mu_l = c 2^(-alpha l), v_l = v 2^(-beta l)
for l >= 1; the drivers must meet their own stopping rules exactly, pick the
level the weak-error test implies, and land within the sampling error of
sum_l mu_l. A run on the CPU oracle (small grids) checks the same rules on
real fields.
"""
import math

import numpy as np
import pytest

from paper_1910_04727_amd import drivers, inputs

MU0, C, ALPHA = 1.0, 0.08, 2.0
V0, V, BETA = 0.2, 0.01, 2.0


def mock(levels_seen=None):
    def solve(jobs):
        out = {}
        for l, xi in jobs.items():
            if levels_seen is not None:
                levels_seen.append((l, xi.shape[0]))
            mu = MU0 if l == 0 else C * 2.0 ** (-ALPHA * l)
            v = V0 if l == 0 else V * 2.0 ** (-BETA * l)
            y = mu + math.sqrt(v) * xi[:, 0]
            out[l] = (y, np.zeros_like(y))
        return out
    return solve


def true_mean(L):
    return MU0 + sum(C * 2.0 ** (-ALPHA * l) for l in range(1, L + 1))


@pytest.mark.parametrize("eps", [2e-2, 5e-3])
def test_mlmc_meets_its_rules(eps):
    seen = []
    r = drivers.mlmc(mock(seen), eps, M=4, config=9, levels_available=8, n_init=32, alpha=ALPHA)
    assert r.converged
    # variance rule: sum V_l / N_l <= eps^2 / 2 with the final estimates
    assert r.var_of_mean <= eps ** 2 / 2 * (1 + 1e-12)
    # optimal allocation: N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum sqrt(V_k C_k)) (or the samples already taken)
    Cl = [4.0 ** l for l in range(r.L + 1)]
    s = sum(math.sqrt(v * c) for v, c in zip(r.V, Cl))
    for l in range(r.L + 1):
        assert r.N[l] >= math.ceil(2 / eps ** 2 * math.sqrt(r.V[l] / Cl[l]) * s)
    # weak-error rule, and L is the first level where it holds (given the estimated means)
    assert abs(r.means[r.L]) / (2 ** ALPHA - 1) < eps / math.sqrt(2)
    for rd in r.rounds[:-1]:
        if all(n >= no for n, no in zip(rd["N"], rd["Nopt"])):
            assert rd["bias"] >= eps / math.sqrt(2)
    # estimate within 5 sigma of the exact mean plus the bias bound
    assert abs(r.mean - true_mean(r.L)) <= 5 * math.sqrt(r.var_of_mean)
    assert abs(true_mean(r.L) - true_mean(60)) <= eps / math.sqrt(2)
    # samples are extended, never replaced: every level's rows were requested once, in order
    assert sum(n for l, n in seen if l == 0) == r.N[0]


def test_mlmc_estimates_rates():
    """beta from the sample variances is sharp; alpha from the level means carries their
    sampling noise (the finest level's mean is only resolved to about its own size)."""
    r = drivers.mlmc(mock(), 2e-3, M=4, config=9, levels_available=8, n_init=256)
    assert r.converged
    assert abs(r.beta - BETA) < 0.3
    assert 1.0 < r.alpha < 4.0


@pytest.mark.parametrize("eps", [1e-2, 2e-3])
def test_mlqmc_meets_its_rules(eps):
    r = drivers.mlqmc(mock(), eps, M=4, config=9, levels_available=8, m_init=4, nshift=8, alpha=ALPHA)
    assert r.converged
    assert r.var_of_mean <= eps ** 2 / 2
    assert abs(r.means[r.L]) / (2 ** ALPHA - 1) < eps / math.sqrt(2)
    assert all(n % 8 == 0 and ((n // 8) & (n // 8 - 1)) == 0 for n in r.N)  # R x 2^m points
    assert abs(r.mean - true_mean(r.L)) <= 6 * math.sqrt(r.var_of_mean) + 1e-12


def test_qmc_needs_fewer_samples_than_mc_on_a_smooth_integrand():
    eps = 2e-3
    mc = drivers.mlmc(mock(), eps, M=4, config=9, levels_available=8, n_init=32, alpha=ALPHA)
    qmc = drivers.mlqmc(mock(), eps, M=4, config=9, levels_available=8, m_init=4, nshift=8, alpha=ALPHA)
    assert sum(qmc.N) < sum(mc.N) / 10


def test_mlmc_on_the_oracle():
    """FMG-MLMC driver on real fields: 8^2 .. 32^2 grids, sigma^2 = 1, corr_len 0.3, 16 modes."""
    from oracle import oracle as O
    cfg = dict(sigma2=1.0, corr_len=0.3, n_modes=16)
    tab = O.kl_table(cfg["sigma2"], cfg["corr_len"], cfg["n_modes"])

    def solve(jobs):
        return {l: O.solve_level(cfg["sigma2"], cfg["corr_len"], tab, 8 << l, l, xi)[:2] for l, xi in jobs.items()}
    r = drivers.mlmc(solve, 2e-2, M=16, config=9, levels_available=3, n_init=32)
    assert r.var_of_mean <= (2e-2) ** 2 / 2 * (1 + 1e-12)
    assert r.L >= 1 and all(n >= 32 for n in r.N)
    # telescoping: Y_0 = Q^f_0, and the level-(l+1) coarse Q equals the level-l fine Q on a shared sample
    xi = inputs.mc_normals_blocked(0, 4, 16, 9, 1)
    f0, _ = solve({0: xi})[0]
    _, c1 = solve({1: xi})[1]
    np.testing.assert_allclose(c1, f0, rtol=1e-11)
