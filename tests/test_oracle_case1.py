"""Pins of the oracle's Case I (Table 1): Dirichlet pressure on all four sides
(west 100, east 0, south 10, north 50, scaled by 1/100), QoI = u(1/2, 1/2).

Facts fixed by the mathematics rather than by the oracle's own formulas:
  - a field invariant under the eight symmetries of the square gives the
    centre pressure (g_W + g_E + g_S + g_N) / 4 exactly (the four boundary
    responses are equal by symmetry and sum to one);
  - equal data on every side reproduce that constant; the discrete maximum
    principle; zero net flux through the boundary;
  - superposition over the four sides;
  - the FMG pass against a dense direct solve, Q^c_l = Q^f_{l-1}, and the
    per-cycle convergence factor.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_04727_amd import inputs

G = O.CASE1_G   # west, east, south, north


def _dense(K):
    n = K.shape[0]
    fc = O.faces(K, case=1)
    A = np.zeros((n * n, n * n))
    for q in range(n * n):
        e = np.zeros(n * n)
        e[q] = 1.0
        A[:, q] = O.apply(K, e.reshape(n, n), fc).ravel()
    return A


def _solve(K, g=G):
    n = K.shape[0]
    b = O.rhs(K, g[0], g[1], case=1, pS=g[2], pN=g[3]).ravel()
    return np.linalg.solve(_dense(K), b).reshape(n, n)


def _d4_symmetric(n, rng, s=1.0):
    """log K averaged over the orbit of each cell under rotations and reflections."""
    g = s * rng.standard_normal((n, n))
    imgs = []
    for k in range(4):
        r = np.rot90(g, k)
        imgs += [r, r.T]
    return np.exp(np.mean(imgs, axis=0))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_symmetric_field_gives_the_mean_of_the_boundary_values(n):
    rng = np.random.default_rng(n)
    K = _d4_symmetric(n, rng, 1.5)
    assert np.allclose(K, K.T) and np.allclose(K, K[::-1, ::-1])
    p = _solve(K)
    assert abs(O.qoi(K, p, case=1) - sum(G) / 4) <= 1e-14
    out = O.fmg_sample(K, level=0 if n == 4 else 1, tol=1e-14, max_cycles=60, case=1)
    assert out["rc"] == 0 and out["flags"] == 0
    assert abs(out["qf"] - sum(G) / 4) <= 1e-13


def test_a_non_symmetric_field_moves_the_centre_value():
    rng = np.random.default_rng(3)
    K = np.exp(rng.standard_normal((8, 8)))
    assert abs(O.qoi(K, _solve(K), case=1) - sum(G) / 4) > 1e-3


def test_equal_data_reproduce_the_constant_and_the_maximum_principle():
    rng = np.random.default_rng(5)
    K = np.exp(2.0 * rng.standard_normal((16, 16)))
    p = _solve(K, (0.7, 0.7, 0.7, 0.7))
    assert np.max(np.abs(p - 0.7)) <= 1e-13
    p = _solve(K)
    assert p.min() >= min(G) - 1e-14 and p.max() <= max(G) + 1e-14


def test_zero_net_boundary_flux():
    rng = np.random.default_rng(7)
    n = 16
    K = np.exp(rng.standard_normal((n, n)))
    p = _solve(K)
    Tx, Ty = O.faces(K, case=1)
    flux = (np.sum(Tx[:, 0] * (G[0] - p[:, 0])) + np.sum(Tx[:, n] * (G[1] - p[:, -1]))
            + np.sum(Ty[0, :] * (G[2] - p[0, :])) + np.sum(Ty[n, :] * (G[3] - p[-1, :])))
    scale = np.sum(Tx[:, 0] * np.abs(G[0] - p[:, 0]))
    assert abs(flux) <= 1e-13 * scale
    # the no-flow faces of Case II are Dirichlet faces here
    assert np.all(Ty[0] > 0) and np.all(Ty[n] > 0)
    assert np.array_equal(Ty[0], 2 * K[0]) and np.array_equal(Ty[n], 2 * K[-1])


def test_superposition_over_the_sides():
    rng = np.random.default_rng(9)
    K = np.exp(rng.standard_normal((8, 8)))
    unit = [O.qoi(K, _solve(K, tuple(float(k == s) for k in range(4))), case=1) for s in range(4)]
    assert abs(sum(unit) - 1.0) <= 1e-14
    assert all(u > 0 for u in unit)
    q = O.qoi(K, _solve(K), case=1)
    assert abs(q - sum(w * g for w, g in zip(unit, G))) <= 1e-14


@pytest.mark.parametrize("n", [8, 16])
def test_fmg_matches_the_dense_solve(n):
    rng = np.random.default_rng(11 + n)
    for _ in range(3):
        K = np.exp(1.5 * rng.standard_normal((n, n)))
        out = O.fmg_sample(K, level=1, tol=1e-14, max_cycles=80, case=1)
        assert out["flags"] == 0
        ref = O.qoi(K, _solve(K), case=1)
        assert abs(out["qf"] - ref) <= 1e-12 * abs(ref)
        # the coarse-mesh QoI is the exact solve on the injected field
        Kc = O.coarsen(K)
        refc = O.qoi(Kc, _solve(Kc), case=1)
        assert abs(out["qc"] - refc) <= 1e-12 * abs(refc)


def test_interpolation_ghosts_reproduce_constants():
    """With equal data c on every side, FMG interpolation of the constant c is c
    everywhere, corners included; a correction is reflected oddly about every
    side (homogeneous Dirichlet), and twice (i.e. evenly) at a corner."""
    xc = np.full((4, 4), 0.3)
    x = O.fmg_interp(xc, 0.3, 0.3, case=1, pS=0.3, pN=0.3)
    assert np.max(np.abs(x - 0.3)) <= 1e-16
    ec = np.random.default_rng(1).standard_normal((4, 4))
    x = O.prolong_add(ec, np.zeros((8, 8)), case=1)
    # fine cells (3, 0) and (0, 0): the ghost row below is -ec[0], the corner ghost +ec[0, 0]
    assert abs(x[0, 3] - (9 * ec[0, 1] + 3 * ec[0, 2] + 3 * (-ec[0, 1]) + (-ec[0, 2])) / 16) <= 1e-15
    assert abs(x[0, 0] - (9 * ec[0, 0] + 3 * (-ec[0, 0]) + 3 * (-ec[0, 0]) + ec[0, 0]) / 16) <= 1e-15


def test_vcycle_factor_below_0p2_case1():
    tab = O.kl_table(1.0, 0.3, 64)
    worst = 0.0
    for lev, n in enumerate([16, 32, 64]):
        xi = inputs.mc_normals(30, 64, config=1, level=lev)
        for s in range(xi.shape[0]):
            K = O.field(n, 0.3, tab, xi[s])
            out = O.fmg_sample(K, level=lev, tol=1e-13, max_cycles=60, history=True, case=1)
            assert out["flags"] == 0
            for h in out["hist"]:
                h = h[h > 1e-13]
                if len(h) > 1:
                    worst = max(worst, float(np.max(h[1:] / h[:-1])))
    assert 0.0 < worst < 0.2, worst


def test_coarse_qoi_is_the_level_below_fine_qoi():
    tab = O.kl_table(1.0, 0.2, 256)
    xi = inputs.mc_normals(6, 256, config=2, level=0)
    lo = O.solve_level(1.0, 0.2, tab, 32, 0, xi, tol=1e-14, max_cycles=80, case=1)
    hi = O.solve_level(1.0, 0.2, tab, 64, 1, xi, tol=1e-14, max_cycles=80, case=1)
    assert np.all(lo[3] == 0) and np.all(hi[3] == 0)
    assert np.max(np.abs(hi[1] - lo[0]) / np.abs(lo[0])) < 1e-11
    # Case I and Case II are different problems on the same fields
    two = O.solve_level(1.0, 0.2, tab, 32, 0, xi, tol=1e-14, max_cycles=80)
    assert np.min(np.abs(two[0] - lo[0])) > 1e-3
