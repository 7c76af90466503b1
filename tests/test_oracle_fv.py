"""Pins of the oracle's finite-volume operator, QoI and multigrid pieces.

Closed forms derived from the continuous problem (Section 3.1, Table 1 Case II)
and the flux balance of the scheme; invariances; brute-force dense solves.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(K):
    """Operator matrix assembled by applying the oracle operator to unit vectors."""
    n = K.shape[0]
    N = n * n
    fc = O.faces(K)
    A = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        A[:, q] = O.apply(K, e.reshape(n, n), fc).ravel()
    return A


def _exact(K, pW=1.0, pE=0.0):
    n = K.shape[0]
    A = _dense(K)
    b = O.rhs(K, pW, pE).ravel()
    return np.linalg.solve(A, b).reshape(n, n)


def _lognormal(n, rng, s=1.0):
    return np.exp(s * rng.standard_normal((n, n)))


def test_operator_symmetric_m_matrix():
    rng = np.random.default_rng(0)
    K = _lognormal(8, rng, 2.0)
    A = _dense(K)
    assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    assert np.all(np.linalg.eigvalsh(A) > 0)
    # weak diagonal dominance, strict on the Dirichlet columns
    rows = np.diag(A) + off.sum(axis=1)
    assert np.all(rows >= -1e-13)
    assert np.all(rows.reshape(8, 8)[:, 0] > 0) and np.all(rows.reshape(8, 8)[:, -1] > 0)


def test_constant_k_linear_pressure():
    """Constant k: p = pW + (pE - pW) x at cell centres exactly, Q = k (pW - pE)."""
    for n in [4, 8, 16]:
        K = np.full((n, n), 3.0)
        p = _exact(K)
        xc = (np.arange(n) + 0.5) / n
        assert np.max(np.abs(p - (1.0 - xc)[None, :])) < 1e-13
        assert abs(O.qoi(K, p) - 3.0) < 1e-13


def test_golden_case2_paper_units():
    """Table 1 Case II with the paper's boundary values u_W = 100, u_E = 0."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "case2_constant_k.txt"))
            if l.strip() and not l.startswith("#")]
    for n, k, pw, pe, q in rows:
        n = int(n)
        K = np.full((n, n), float(k))
        p = _exact(K, float(pw), float(pe))
        assert abs(O.qoi(K, p, float(pe)) - float(q)) <= 1e-12 * abs(float(q))


def test_layered_closed_forms():
    """y-layered k_j: rows are independent, Q = h sum_j k_j (pW - pE).
    x-layered k_i: resistances in series, Q = 1 / (h sum_i 1/k_i)."""
    rng = np.random.default_rng(1)
    n = 8
    h = 1.0 / n
    ky = np.exp(rng.standard_normal(n))
    K = np.repeat(ky[:, None], n, axis=1)
    assert abs(O.qoi(K, _exact(K)) - h * ky.sum()) < 1e-13 * ky.sum()
    kx = np.exp(rng.standard_normal(n))
    K = np.repeat(kx[None, :], n, axis=0)
    ref = 1.0 / (h * np.sum(1.0 / kx))
    assert abs(O.qoi(K, _exact(K)) - ref) < 1e-13 * ref


def test_flux_balance_and_invariances():
    rng = np.random.default_rng(2)
    n = 8
    K = _lognormal(n, rng, 1.5)
    p = _exact(K)
    q = O.qoi(K, p)
    inflow = np.sum(2.0 * K[:, 0] * (1.0 - p[:, 0]))
    assert abs(inflow - q) < 1e-13 * abs(q)
    # mirror in y: same Q
    assert abs(O.qoi(K[::-1], _exact(K[::-1])) - q) < 1e-13 * abs(q)
    # mirror in x with swapped Dirichlet data: Q -> -Q
    Kx = K[:, ::-1]
    assert abs(O.qoi(Kx, _exact(Kx, 0.0, 1.0), 1.0) + q) < 1e-13 * abs(q)
    # linear in k
    assert abs(O.qoi(7.0 * K, _exact(7.0 * K)) - 7.0 * q) < 1e-13 * abs(q)


def test_residual_of_exact_solution_vanishes():
    rng = np.random.default_rng(3)
    K = _lognormal(8, rng)
    p = _exact(K)
    b = O.rhs(K)
    assert np.max(np.abs(O.residual(K, b, p))) < 1e-13


def test_gauss_seidel_fixed_point_and_energy():
    """The exact solution is a fixed point of both half-sweeps; each half-sweep
    lowers the A-norm of the error and only touches its own colour."""
    rng = np.random.default_rng(4)
    n = 8
    K = _lognormal(n, rng)
    A = _dense(K)
    b = O.rhs(K)
    p = _exact(K)
    for c in (0, 1):
        assert np.max(np.abs(O.rbgs_half(K, b, p, c) - p)) < 1e-13
    x = rng.standard_normal((n, n))
    colour = (np.add.outer(np.arange(n), np.arange(n)) % 2)
    for c in (0, 1, 0, 1):
        e0 = (x - p).ravel()
        y = O.rbgs_half(K, b, x, c)
        assert np.array_equal(y[colour != c], x[colour != c])
        e1 = (y - p).ravel()
        assert e1 @ A @ e1 < e0 @ A @ e0
        x = y


def test_transfer_operators():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((8, 8))
    rc = O.restrict(r)
    assert abs(rc.sum() - r.sum()) < 1e-12                 # integrated residual conserved
    assert abs(rc[1, 2] - r[2:4, 4:6].sum()) < 1e-15
    # bilinear interpolation reproduces functions linear in x and y away from the
    # Dirichlet sides, and exactly everywhere for data matching the Dirichlet values
    nc = 4
    xc = (np.arange(nc) + 0.5) / nc
    xf = (np.arange(2 * nc) + 0.5) / (2 * nc)
    lin_c = np.repeat((1.0 - xc)[None, :], nc, axis=0)
    assert np.max(np.abs(O.fmg_interp(lin_c, 1.0, 0.0) - (1.0 - xf)[None, :])) < 1e-15
    yc = xc
    yf = xf
    f_c = np.repeat((2.0 + yc)[:, None], nc, axis=1)
    f_f = np.repeat((2.0 + yf)[:, None], 2 * nc, axis=1)
    got = O.prolong_add(f_c, np.zeros((2 * nc, 2 * nc)))
    assert np.max(np.abs(got[1:-1, 1:-1] - f_f[1:-1, 1:-1])) < 1e-15
    # homogeneous Dirichlet correction: a constant decays to 3/4 in the boundary columns
    one = O.prolong_add(np.ones((nc, nc)), np.zeros((2 * nc, 2 * nc)))
    assert np.allclose(one[:, 1:-1], 1.0) and np.allclose(one[:, [0, -1]], 0.5)


def test_coarsest_direct_solve():
    rng = np.random.default_rng(6)
    K = _lognormal(4, rng, 2.0)
    b = rng.standard_normal((4, 4))
    x = O.chol_solve(K, b)
    ref = np.linalg.solve(_dense(K), b.ravel()).reshape(4, 4)
    assert np.max(np.abs(x - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_fmg_matches_dense_solve(n):
    """Brute force: FMG to tol 3e-15 vs a dense LU solve of the same operator.

    (The QoI error is up to ~100x the relative residual on these grids, so the
    solve is driven close to the FP64 floor.)"""
    rng = np.random.default_rng(100 + n)
    for level in ((0, 1) if n > 4 else (0,)):
        for _ in range(4):
            K = _lognormal(n, rng, 1.5)
            out = O.fmg_sample(K, level=level, tol=3e-15, max_cycles=100)
            assert out["flags"] == 0
            q = O.qoi(K, _exact(K))
            assert abs(out["qf"] - q) <= 1e-12 * abs(q)
            if level == 1:
                Kc = O.coarsen(K)
                qc = O.qoi(Kc, _exact(Kc))
                assert abs(out["qc"] - qc) <= 1e-12 * abs(qc)
            else:
                assert out["qc"] == 0.0


def test_fmg_rejects_level_without_coarse_stage():
    K = np.ones((4, 4))
    assert O.fmg_sample(K, level=1)["rc"] == -1
