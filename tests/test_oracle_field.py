"""Pins of the oracle's field synthesis and coarsening (Sections 2.5 and 3.1 (2))."""
import numpy as np
import pytest

from oracle import oracle as O


def test_coarsening_is_level_below_bitwise():
    """Injection k^c_{I,J} = k^f_{2I,2J} of the corner-sampled field is exactly
    the field synthesised on the coarse grid (h is a power of two)."""
    tab = O.kl_table(1.0, 0.2, 256)
    rng = np.random.default_rng(3)
    for _ in range(3):
        xi = rng.standard_normal(256)
        Kf = O.field(64, 0.2, tab, xi)
        for n in [32, 16, 8, 4]:
            Kc = O.field(n, 0.2, tab, xi)
            Kf = O.coarsen(Kf)
            assert np.array_equal(Kf, Kc)


def test_truncated_covariance_converges_to_kernel():
    """sum_m lambda_m phi_m(x) phi_m(x') built from unit-vector fields -> sigma^2 e^{-|dx|/l - |dy|/l}.

    With xi = e_m the synthesised log-field is sqrt(lambda_m) phi_m, so the sum of
    products over m is the truncated covariance. Off the diagonal it must approach
    the separable exponential kernel as M grows.
    """
    sigma2, corr_len, n = 1.0, 0.3, 8
    M = 3000
    tab = O.kl_table(sigma2, corr_len, M)
    G = np.zeros((M, n * n))
    for m in range(M):
        e = np.zeros(M)
        e[m] = 1.0
        G[m] = np.log(O.field(n, corr_len, tab, e)).ravel()
    Cm = G.T @ G
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    X = X.ravel()
    Y = Y.ravel()
    Cex = sigma2 * np.exp(-(np.abs(X[:, None] - X[None, :]) + np.abs(Y[:, None] - Y[None, :])) / corr_len)
    off = ~np.eye(n * n, dtype=bool)
    assert np.max(np.abs(Cm - Cex)[off]) < 0.02
    # diagonal: variance sigma^2 up to truncation, never above it
    d = np.diag(Cm)
    assert np.all(d <= sigma2 + 1e-12) and np.all(d > 0.9 * sigma2)


def test_sample_variance_matches_truncated_kl():
    """Monte Carlo pointwise variance of g over S samples vs the KL variance,
    within the chi-square sampling band sqrt(2/(S-1)) (5 sigma)."""
    sigma2, corr_len, M, n, S = 1.0, 0.3, 64, 8, 4000
    tab = O.kl_table(sigma2, corr_len, M)
    rng = np.random.default_rng(11)
    G = np.array([np.log(O.field(n, corr_len, tab, rng.standard_normal(M))).ravel() for _ in range(S)])
    var = G.var(axis=0, ddof=1)
    unit = np.zeros((M, n * n))
    for m in range(M):
        e = np.zeros(M)
        e[m] = 1.0
        unit[m] = np.log(O.field(n, corr_len, tab, e)).ravel()
    var_kl = (unit ** 2).sum(axis=0)
    assert np.all(np.abs(var / var_kl - 1.0) < 5 * np.sqrt(2.0 / (S - 1)))
    assert np.all(np.abs(G.mean(axis=0)) < 5 * np.sqrt(var_kl / S))


def test_spatial_mean_variance_is_captured_fraction():
    """Orthonormality: the grid average of sum_m lambda_m phi_a^2 phi_b^2 -> sum_m lambda_m
    (the corner rule for smooth integrands converges at O(h))."""
    sigma2, corr_len, M, n = 1.0, 0.3, 64, 256
    tab = O.kl_table(sigma2, corr_len, M)
    acc = np.zeros((n, n))
    for m in range(M):
        e = np.zeros(M)
        e[m] = 1.0
        acc += np.log(O.field(n, corr_len, tab, e)) ** 2
    assert abs(acc.mean() - tab[2].sum()) < 0.02
