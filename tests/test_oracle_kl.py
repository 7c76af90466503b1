"""Pins of the oracle's Karhunen-Loeve expansion (Section 3.1 (2)).

Each check is independent of the oracle's own formulas: the eigenpairs are
checked against the integral equation they must solve (numerical quadrature),
orthonormality, the trace identity the paper states, the covariance function
itself (Mercer), and a brute-force selection of the 2-D table.
"""
import numpy as np
import pytest

from oracle import oracle as O

CASES = [0.3, 0.2, 0.1, 0.05]


def _gl(a, b, m):
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


@pytest.mark.parametrize("corr_len", CASES)
def test_integral_equation(corr_len):
    """int_0^1 exp(-|s-t|/l) phi_n(t) dt = theta_n phi_n(s), quadrature split at s."""
    c = 1.0 / corr_len
    w, th = O.kl_1d(corr_len, 40)
    for n in [1, 2, 3, 8, 17, 40]:
        for s in [0.0, 0.137, 0.5, 0.81, 1.0 - 2.0 ** -10]:
            acc = 0.0
            for (a, b) in [(0.0, s), (s, 1.0)]:
                if b - a <= 0:
                    continue
                t, wt = _gl(a, b, 120)
                acc += np.sum(wt * np.exp(-c * np.abs(s - t)) * O.kl_phi(n, w[n - 1], t))
            lhs = acc
            rhs = th[n - 1] * O.kl_phi(n, w[n - 1], [s])[0]
            assert abs(lhs - rhs) <= 1e-12, (n, s, lhs, rhs)


@pytest.mark.parametrize("corr_len", CASES)
def test_orthonormal(corr_len):
    w, _ = O.kl_1d(corr_len, 30)
    t, wt = _gl(0.0, 1.0, 200)
    Phi = np.array([O.kl_phi(n, w[n - 1], t) for n in range(1, 31)])
    G = (Phi * wt) @ Phi.T
    assert np.max(np.abs(G - np.eye(30))) <= 1e-13


@pytest.mark.parametrize("corr_len", CASES)
def test_trace_identity(corr_len):
    """sum_n theta_n = sigma^2 meas(Omega) = 1 (Section 3.1 (2)); eigenvalues descend.

    theta_n <= 2c/(c^2 + ((n-1) pi)^2) bounds the tail beyond N by 2c/(pi^2 (N-1)).
    """
    c = 1.0 / corr_len
    N = 4000
    _, th = O.kl_1d(corr_len, N)
    assert np.all(np.diff(th) < 0)
    tail = 1.0 - np.sum(th)
    assert 0.0 < tail <= 2.0 * c / (np.pi ** 2 * (N - 1))


def test_mercer_1d():
    """sum_n theta_n phi_n(s) phi_n(t) -> exp(-c|s-t|) away from the diagonal."""
    corr_len = 0.3
    c = 1.0 / corr_len
    N = 3000
    w, th = O.kl_1d(corr_len, N)
    for s, t in [(0.1, 0.4), (0.5, 0.55), (0.0, 1.0), (0.25, 0.75)]:
        acc = sum(th[k] * O.kl_phi(k + 1, w[k], [s])[0] * O.kl_phi(k + 1, w[k], [t])[0]
                  for k in range(N))
        assert abs(acc - np.exp(-c * abs(s - t))) < 2e-3


def _brute_table(sigma2, corr_len, M):
    _, th = O.kl_1d(corr_len, M)
    pairs = [(-(sigma2 * (th[a] * th[b])), a, b) for a in range(M) for b in range(M)]
    pairs.sort()
    return pairs[:M]


@pytest.mark.parametrize("sigma2,corr_len,M", [(1.0, 0.3, 64), (1.0, 0.2, 256), (2.0, 0.1, 512)])
def test_table_is_top_m(sigma2, corr_len, M):
    a, b, lam = O.kl_table(sigma2, corr_len, M)
    ref = _brute_table(sigma2, corr_len, M)
    assert [(int(x), int(y)) for x, y in zip(a, b)] == [(p[1], p[2]) for p in ref]
    assert np.array_equal(lam, np.array([-p[0] for p in ref]))


def test_table_exact_tie_split():
    """cfg3 (corr 0.1, M=512): the 512th/513th modes are the exact pair (4,29)/(29,4).

    The eigenvalue products are bitwise equal; the (a asc, b asc) tie rule keeps
    (4,29) and drops (29,4).
    """
    a, b, lam = O.kl_table(2.0, 0.1, 513)
    assert (int(a[511]), int(b[511])) == (4, 29)
    assert (int(a[512]), int(b[512])) == (29, 4)
    assert lam[511] == lam[512]
    a2, b2, _ = O.kl_table(2.0, 0.1, 512)
    assert (int(a2[-1]), int(b2[-1])) == (4, 29)


@pytest.mark.parametrize("sigma2,corr_len,M,frac", [(1.0, 0.3, 64, 0.8661), (1.0, 0.2, 256, 0.9104),
                                                    (2.0, 0.1, 512, 0.8650), (3.0, 0.05, 1024, 0.7998)])
def test_captured_variance(sigma2, corr_len, M, frac):
    """Captured fraction sum_m lambda_m / sigma^2 (the paper's 99% rule is replaced by fixed M)."""
    _, _, lam = O.kl_table(sigma2, corr_len, M)
    assert abs(lam.sum() / sigma2 - frac) < 5e-5
