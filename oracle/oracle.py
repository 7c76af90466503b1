"""ctypes wrapper around the plain-C FP64 oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.
Every function cites, in oracle.c, the passage of the paper it follows.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_pd = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_pi = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_pl = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build
            build.build()
        L = C.CDLL(path)
        sig = {
            "oracle_kl_root": (_d, [_d, _i]),
            "oracle_kl_theta": (_d, [_d, _d]),
            "oracle_kl_phi": (_d, [_i, _d, _d]),
            "oracle_kl_1d": (None, [_d, _i, _pd, _pd]),
            "oracle_kl_table": (_i, [_d, _d, _i, _pi, _pi, _pd]),
            "oracle_field": (None, [_i, _d, _i, _pi, _pi, _pd, _pd, _pd]),
            "oracle_coarsen": (None, [_i, _pd, _pd]),
            "oracle_faces": (None, [_i, _pd, _i, _pd, _pd]),
            "oracle_apply": (None, [_i, _pd, _pd, _pd, _pd]),
            "oracle_rhs": (None, [_i, _pd, _pd, _pd, _i, _pd]),
            "oracle_residual": (None, [_i, _pd, _pd, _pd, _pd, _pd]),
            "oracle_qoi": (_d, [_i, _pd, _pd, _pd, _i]),
            "oracle_rbgs_half": (None, [_i, _pd, _pd, _pd, _pd, _i]),
            "oracle_restrict": (None, [_i, _pd, _pd]),
            "oracle_prolong_add": (None, [_i, _pd, _i, _pd]),
            "oracle_fmg_interp": (None, [_i, _pd, _pd, _i, _pd]),
            "oracle_chol_factor": (_i, [_i, _pd, _pd, _pd]),
            "oracle_chol_solve": (None, [_i, _pd, _pd, _pd]),
            "oracle_coarsen_faces": (None, [_i, _pd, _pd, _pd, _pd]),
            "oracle_fmg_sample": (_i, [_i, _i, _i, _pd, _pd, _i, _d, _i, _i, _i, _i,
                                       C.POINTER(_d), C.POINTER(_d), _pi, C.POINTER(_i), C.c_void_p]),
            "oracle_solve_level": (_i, [_d, _d, _i, _pi, _pi, _pd, _i, _i, _i, _i64, _pd, _pd, _i,
                                        _d, _i, _i, _i, _i, _pd, _pd, _pi, _pi, _i]),
            "oracle_max_threads": (_i, []),
            "oracle_sum": (_d, [_i64, _pd]),
            "oracle_level_stats": (_i, [_i64, _pd, _pd, _pd]),
            "oracle_rqmc_stats": (_i, [_i64, _i, _pd, _pd, _pd, C.c_void_p]),
            "oracle_optimal_nl": (None, [_i, _pd, _pd, _d, _pl]),
            "oracle_cnn_nparams": (_i64, [_i, _i, _i]),
            "oracle_cnn_forward": (None, [_i, _i, _i, _i, _i, _pd, _pd, _pd, C.c_void_p, C.c_void_p]),
            "oracle_cnn_loss_grad": (_d, [_i, _i, _i, _i, _i, _pd, _pd, _pd, _pd]),
            "oracle_cnn_loss_grad_kind": (_d, [_i, _i, _i, _i, _i, _pd, _pd, C.c_void_p, _i, _pd]),
            "oracle_adam": (None, [_i64, _pd, _pd, _pd, _pd, _i, _d, _d, _d, _d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- Karhunen-Loeve -------------------------------------------------------
def kl_1d(corr_len, count):
    w = np.zeros(count)
    th = np.zeros(count)
    lib().oracle_kl_1d(corr_len, count, w, th)
    return w, th


def kl_phi(n, w, s):
    """Normalised 1-D eigenfunction number n (1-based) at points s."""
    f = lib().oracle_kl_phi
    return np.array([f(int(n), float(w), float(x)) for x in np.atleast_1d(s)])


def kl_table(sigma2, corr_len, M):
    a = np.zeros(M, np.int32)
    b = np.zeros(M, np.int32)
    lam = np.zeros(M)
    rc = lib().oracle_kl_table(sigma2, corr_len, M, a, b, lam)
    if rc != 0:
        raise ValueError("oracle_kl_table failed")
    return a, b, lam


def field(n, corr_len, table, xi):
    a, b, lam = table
    K = np.zeros((n, n))
    lib().oracle_field(n, corr_len, len(a), a, b, lam, _f64(xi), K)
    return K


def coarsen(Kf):
    n = Kf.shape[0]
    Kc = np.zeros((n // 2, n // 2))
    lib().oracle_coarsen(n, _f64(Kf), Kc)
    return Kc


# --- finite volumes ------------------------------------------------------
# Boundary case of Table 1: 2 = Case II (Dirichlet west/east, no flow south/north,
# east outflow), 1 = Case I (Dirichlet on all sides, centre pressure). Boundary
# values (west, east, south, north); the Case I defaults are the paper's
# 100/0/10/50 scaled by 1/100, as Case II's 1/0 is its 100/0.
CASE1_G = (1.0, 0.0, 0.1, 0.5)


def _g(pW, pE, pS=0.0, pN=0.0):
    return np.array([pW, pE, pS, pN], dtype=np.float64)


def faces(K, case=2):
    n = K.shape[0]
    Tx = np.zeros((n, n + 1))
    Ty = np.zeros((n + 1, n))
    lib().oracle_faces(n, _f64(K), int(case), Tx, Ty)
    return Tx, Ty


def apply(K, x, fc=None, case=2):
    n = K.shape[0]
    Tx, Ty = fc if fc is not None else faces(K, case)
    y = np.zeros((n, n))
    lib().oracle_apply(n, Tx, Ty, _f64(x), y)
    return y


def rhs(K, pW=1.0, pE=0.0, case=2, pS=0.0, pN=0.0):
    n = K.shape[0]
    Tx, Ty = faces(K, case)
    b = np.zeros((n, n))
    lib().oracle_rhs(n, Tx, Ty, _g(pW, pE, pS, pN), int(case), b)
    return b


def residual(K, b, x, case=2):
    n = K.shape[0]
    Tx, Ty = faces(K, case)
    r = np.zeros((n, n))
    lib().oracle_residual(n, Tx, Ty, _f64(b), _f64(x), r)
    return r


def qoi(K, x, pE=0.0, case=2):
    n = K.shape[0]
    Tx, _ = faces(K, case)
    return lib().oracle_qoi(n, Tx, _f64(x), _g(0.0, pE), int(case))


def rbgs_half(K, b, x, colour, case=2):
    n = K.shape[0]
    Tx, Ty = faces(K, case)
    x = _f64(x).copy()
    lib().oracle_rbgs_half(n, Tx, Ty, _f64(b), x, colour)
    return x


def restrict(r):
    n = r.shape[0]
    rc = np.zeros((n // 2, n // 2))
    lib().oracle_restrict(n, _f64(r), rc)
    return rc


def prolong_add(ec, x, case=2):
    x = _f64(x).copy()
    lib().oracle_prolong_add(ec.shape[0], _f64(ec), int(case), x)
    return x


def fmg_interp(xc, pW=1.0, pE=0.0, case=2, pS=0.0, pN=0.0):
    nc = xc.shape[0]
    x = np.zeros((2 * nc, 2 * nc))
    lib().oracle_fmg_interp(nc, _f64(xc), _g(pW, pE, pS, pN), int(case), x)
    return x


def chol_solve(K, b, case=2):
    n = K.shape[0]
    Tx, Ty = faces(K, case)
    L = np.zeros((n * n, n * n))
    if lib().oracle_chol_factor(n, Tx, Ty, L) != 0:
        raise ValueError("not positive definite")
    x = np.zeros(n * n)
    lib().oracle_chol_solve(n * n, L, _f64(b).ravel(), x)
    return x.reshape(n, n)


# --- full multigrid ------------------------------------------------------
W_MAX = 64  # coarse grids with n <= 64 get W-cycle (two) coarse-grid corrections


def boundary(case, pW=None, pE=None, pS=None, pN=None):
    """(g[4], case) with the defaults of the case filled in."""
    d = CASE1_G if case == 1 else (1.0, 0.0, 0.0, 0.0)
    v = [d[k] if x is None else float(x) for k, x in enumerate((pW, pE, pS, pN))]
    if case not in (1, 2):
        raise ValueError("case must be 1 or 2")
    return _g(*v), int(case)


def fmg_sample(K, level, tol=1e-10, max_cycles=50, nu1=2, nu2=2, pW=None, pE=None,
               n_coarsest=4, history=False, wmax=W_MAX, case=2, pS=None, pN=None):
    """One FMG pass; returns dict(qf, qc, cycles, flags[, hist])."""
    g, cs = boundary(case, pW, pE, pS, pN)
    n = K.shape[0]
    qf = C.c_double()
    qc = C.c_double()
    cyc = np.zeros(2, np.int32)
    fl = C.c_int()
    hist = np.zeros(2 * max_cycles) if history else None
    rc = lib().oracle_fmg_sample(n, n_coarsest, level, _f64(K), g, cs, tol, max_cycles,
                                 nu1, nu2, wmax, C.byref(qf), C.byref(qc), cyc, C.byref(fl),
                                 hist.ctypes.data if history else None)
    out = dict(qf=qf.value, qc=qc.value, cycles=cyc, flags=fl.value, rc=rc)
    if history:
        out["hist"] = hist.reshape(2, max_cycles)
    return out


def solve_level(sigma2, corr_len, table, n_fine, level, xi, tol=1e-10, max_cycles=50,
                nu1=2, nu2=2, pW=None, pE=None, n_coarsest=4, nthreads=0, wmax=W_MAX, case=2,
                pS=None, pN=None):
    """Batched oracle: xi [ns, M] -> qf, qc [ns], cycles [ns, 2], flags [ns]."""
    g, cs = boundary(case, pW, pE, pS, pN)
    a, b, lam = table
    xi = _f64(xi)
    ns = xi.shape[0]
    qf = np.zeros(ns)
    qc = np.zeros(ns)
    cyc = np.zeros((ns, 2), np.int32)
    fl = np.zeros(ns, np.int32)
    rc = lib().oracle_solve_level(sigma2, corr_len, len(a), a, b, lam, n_fine, n_coarsest,
                                  level, ns, xi, g, cs, tol, max_cycles, nu1, nu2, wmax, qf, qc,
                                  cyc, fl, nthreads)
    if rc != 0:
        raise RuntimeError("oracle_solve_level failed")
    return qf, qc, cyc, fl


def max_threads():
    return lib().oracle_max_threads()


# --- estimators ----------------------------------------------------------
def comp_sum(v):
    v = _f64(v)
    return lib().oracle_sum(v.size, v)


def level_stats(qf, qc):
    out = np.zeros(5)
    lib().oracle_level_stats(len(qf), _f64(qf), _f64(qc), out)
    return dict(mean_y=out[0], var_y=out[1], mean_qf=out[2], var_qf=out[3], mean_qc=out[4])


def rqmc_stats(qf, qc, nshift):
    qf = _f64(qf)
    qc = _f64(qc)
    npts = qf.size // nshift
    out = np.zeros(2)
    sm = np.zeros(nshift)
    lib().oracle_rqmc_stats(npts, nshift, qf, qc, out, sm.ctypes.data)
    return dict(mean_y=out[0], var_mean=out[1], shift_means=sm)


def optimal_nl(V, Cst, eps):
    V = _f64(V)
    Cst = _f64(Cst)
    N = np.zeros(len(V), np.int64)
    lib().oracle_optimal_nl(len(V), V, Cst, eps, N)
    return N


# --- learned warm start (oracle/cnn.c) ------------------------------------
CNN_CIN, CNN_WIDTH, CNN_RES = 2, 32, 4


def cnn_nparams(cin=CNN_CIN, F=CNN_WIDTH, R=CNN_RES):
    return int(lib().oracle_cnn_nparams(cin, F, R))


def cnn_forward(theta, x, cin=CNN_CIN, F=CNN_WIDTH, R=CNN_RES, acts=False):
    """x [B][cin][n][n] -> y [B][n][n] (and z, h [B][R+1][F][n][n] if acts)."""
    x = _f64(x)
    B, n = x.shape[0], x.shape[-1]
    y = np.zeros((B, n, n))
    z = np.zeros((B, R + 1, F, n, n)) if acts else None
    h = np.zeros((B, R + 1, F, n, n)) if acts else None
    lib().oracle_cnn_forward(n, B, cin, F, R, _f64(theta), x, y,
                             z.ctypes.data if acts else None, h.ctypes.data if acts else None)
    return (y, z, h) if acts else y


def cnn_loss_grad(theta, x, t, cin=CNN_CIN, F=CNN_WIDTH, R=CNN_RES):
    x = _f64(x)
    B, n = x.shape[0], x.shape[-1]
    g = np.zeros(cnn_nparams(cin, F, R))
    L = lib().oracle_cnn_loss_grad(n, B, cin, F, R, _f64(theta), x, _f64(t), g)
    return L, g


def cnn_residual_loss_grad(theta, x, cin=CNN_CIN, F=CNN_WIDTH, R=CNN_RES):
    """Residual loss mean((x1 - A y)^2), A from K = exp(x0); returns (L, grad)."""
    x = _f64(x)
    B, n = x.shape[0], x.shape[-1]
    g = np.zeros(cnn_nparams(cin, F, R))
    L = lib().oracle_cnn_loss_grad_kind(n, B, cin, F, R, _f64(theta), x, None, 1, g)
    return L, g


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on theta, m, v (float64 arrays)."""
    lib().oracle_adam(theta.size, theta, _f64(g), m, v, t, lr, beta1, beta2, eps)
