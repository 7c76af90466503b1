"""Thin ctypes binding of the C ABI in include/fmgmc.h (argument marshalling only).

Every step of the method runs in the HIP library libfmgmc.so; this module only
converts arguments. Arrays may be torch tensors (device or host) or numpy
arrays (host). If the library has not been built the import of this module
succeeds but every call raises: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmgmc.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, ENONFINITE = 0, -1, -2, -3, -4, -5
FLAG_NOTCONV, FLAG_NONFINITE, FLAG_FP64, FLAG_WARM_REJECTED = 1, 2, 4, 8
SOLVERS = {"fp64": 0, "fp32_ir": 1}
KL_PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp64_dense": 3}


class Field(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("corr_len", C.c_double), ("n_modes", C.c_int32),
                ("cov_kind", C.c_int32)]


class Hier(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n0", C.c_int32), ("n_coarsest", C.c_int32),
                ("boundary", C.c_int32), ("p_west", C.c_double), ("p_east", C.c_double),
                ("p_south", C.c_double), ("p_north", C.c_double)]


# Table 1: case 2 (Dirichlet west/east, no flow south/north, east outflow) and
# case 1 (Dirichlet on every side, centre pressure). Default boundary values
# (west, east, south, north): the paper's 100/0 and 100/0/10/50 scaled by 1/100
# (the problem is linear in them).
BOUNDARY_DEFAULTS = {2: (1.0, 0.0, 0.0, 0.0), 1: (1.0, 0.0, 0.1, 0.5)}


class Opts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("kl_prec", C.c_int32), ("nu1", C.c_int32),
                ("nu2", C.c_int32), ("max_cycles", C.c_int32), ("inner_cycles", C.c_int32),
                ("max_batch", C.c_int32), ("w_max_n", C.c_int32), ("rel_tol", C.c_double),
                ("inner_first", C.c_int32), ("separate_coarse", C.c_int32), ("fuse_cycles", C.c_int32),
                ("warm", C.c_int32), ("warm_min_n", C.c_int32), ("warm_max_n", C.c_int32),
                ("cnn_weights", C.c_char_p),
                ("tune_cache", C.c_char_p)]


class LevelEst(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean_y", C.c_double), ("var_y", C.c_double),
                ("mean_qf", C.c_double), ("var_qf", C.c_double), ("mean_qc", C.c_double)]


MAX_LEVELS = 16


class Est(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("level", LevelEst * MAX_LEVELS), ("mean", C.c_double),
                ("var_of_mean", C.c_double)]


class FmgmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fmgmc error {code}: {msg}")
        self.code = code


_lib = None

_VP = C.c_void_p
_SIGS = {
    "fmgmc_create": (C.c_int, [C.POINTER(_VP), C.POINTER(Field), C.POINTER(Hier), C.POINTER(Opts), C.c_int]),
    "fmgmc_destroy": (C.c_int, [_VP]),
    "fmgmc_mode_table": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32]),
    "fmgmc_kl_modes": (C.c_int, [C.c_double, C.c_double, C.c_int32, _VP, _VP, _VP]),
    "fmgmc_synthesize_field": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP, _VP]),
    "fmgmc_solve_level": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "fmgmc_estimate": (C.c_int, [C.c_int32, _VP, _VP, _VP, C.c_int32, C.POINTER(Est)]),
    "fmgmc_estimate_levels": (C.c_int, [C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "fmgmc_estimate_levels_noalloc": (C.c_int, [C.c_int32, _VP, _VP, _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "fmgmc_solve_levels": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "fmgmc_autotune": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP]),
    "fmgmc_set_schedule": (C.c_int, [_VP, C.c_int32, _VP]),
    "fmgmc_get_schedule": (C.c_int, [_VP, C.c_int32, _VP]),
    "fmgmc_profile_enable": (C.c_int, [_VP, C.c_int32]),
    "fmgmc_profile_read": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP]),
    "fmgmc_cnn_create": (C.c_int, [C.POINTER(_VP), C.c_uint64, C.c_int32]),
    "fmgmc_cnn_destroy": (C.c_int, [_VP]),
    "fmgmc_cnn_get_params": (C.c_int, [_VP, _VP]),
    "fmgmc_cnn_set_params": (C.c_int, [_VP, _VP]),
    "fmgmc_cnn_save": (C.c_int, [_VP, C.c_char_p]),
    "fmgmc_cnn_load": (C.c_int, [_VP, C.c_char_p]),
    "fmgmc_cnn_forward": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP, C.c_int32, _VP]),
    "fmgmc_cnn_grad": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP, C.c_int32, C.POINTER(C.c_double), _VP,
                                 _VP]),
    "fmgmc_cnn_adam": (C.c_int, [_VP, C.c_double, _VP]),
    "fmgmc_cnn_make_data": (C.c_int, [_VP, C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "fmgmc_cnn_train": (C.c_int, [_VP, _VP, C.c_int32, C.c_int64, _VP, C.c_int32, C.c_double, _VP]),
    "fmgmc_set_warm_start": (C.c_int, [_VP, _VP, C.c_int32]),
    "fmgmc_set_warm_range": (C.c_int, [_VP, _VP, C.c_int32, C.c_int32]),
    "fmgmc_last_error": (C.c_char_p, []),
    "fmgmc_version": (C.c_int, []),
}


def lib():
    """Loads libfmgmc.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FmgmcError(EINVAL, f"{LIB_PATH} is missing: build it with paper_1910_04727_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().fmgmc_last_error().decode()


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise FmgmcError(rc, last_error())
    return rc


def _ptr(a):
    """Raw pointer of a torch tensor or numpy array (must be contiguous)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    raise TypeError(f"unsupported array type {type(a)}")


def _stream_ptr(stream):
    if stream is None:
        return None
    return getattr(stream, "cuda_stream", stream)


def kl_modes(sigma2, corr_len, n_modes):
    """Host-only KL mode table: (a, b, lambda) numpy arrays."""
    a = np.zeros(n_modes, np.int32)
    b = np.zeros(n_modes, np.int32)
    lam = np.zeros(n_modes)
    _check(lib().fmgmc_kl_modes(sigma2, corr_len, n_modes, _ptr(a), _ptr(b), _ptr(lam)))
    return a, b, lam


class Context:
    """One library context (field, level hierarchy, solver options) on one device."""

    def __init__(self, sigma2, corr_len, n_modes, n_levels, n0, solver="fp64", kl_prec="fp64",
                 nu1=2, nu2=2, max_cycles=50, inner_cycles=1, max_batch=0, rel_tol=1e-10,
                 p_west=None, p_east=None, device=0, w_max_n=64, inner_first=0, separate_coarse=False,
                 case=2, p_south=None, p_north=None, fuse_cycles=True, cnn_weights=None, warm_min_n=0,
                 warm_max_n=0, tune_cache=None):
        if case not in BOUNDARY_DEFAULTS:
            raise ValueError("case must be 1 or 2 (Table 1)")
        g = [d if v is None else float(v) for d, v in zip(BOUNDARY_DEFAULTS[case], (p_west, p_east, p_south, p_north))]
        self.case = case
        self.field = Field(sigma2, corr_len, n_modes, 0)
        self.hier = Hier(n_levels, n0, 4, 1 if case == 1 else 0, *g)
        self.opts = Opts(SOLVERS[solver], KL_PREC[kl_prec], nu1, nu2, max_cycles, inner_cycles,
                         max_batch, w_max_n, rel_tol, inner_first, 1 if separate_coarse else 0,
                         1 if fuse_cycles else 0, 1 if cnn_weights is not None else 0, warm_min_n, warm_max_n,
                         None if cnn_weights is None else os.fsencode(cnn_weights),
                         None if tune_cache is None else os.fsencode(tune_cache))
        self.n_modes = n_modes
        self.n0 = n0
        self.n_levels = n_levels
        h = _VP()
        _check(lib().fmgmc_create(C.byref(h), C.byref(self.field), C.byref(self.hier),
                                  C.byref(self.opts), device))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().fmgmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    PROF_KINDS = ("pre", "post", "ir", "kl", "small", "cnn", "fused", "irpre")

    def profile(self, enable=True):
        _check(lib().fmgmc_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kind: (ms, launches, algorithmic bytes or flops)}; clears the records."""
        out = {}
        for k, name in enumerate(self.PROF_KINDS):
            ms = C.c_double()
            cnt = C.c_int64()
            alg = C.c_double()
            _check(lib().fmgmc_profile_read(self._h, k, C.byref(ms), C.byref(cnt), C.byref(alg)))
            out[name] = (ms.value, cnt.value, alg.value)
        return out

    def grid(self, level):
        return self.n0 << level

    def mode_table(self):
        a = np.zeros(self.n_modes, np.int32)
        b = np.zeros(self.n_modes, np.int32)
        lam = np.zeros(self.n_modes)
        m = _check_count(lib().fmgmc_mode_table(self._h, _ptr(a), _ptr(b), _ptr(lam), self.n_modes))
        return a[:m], b[:m], lam[:m]

    def synthesize_field(self, level, xi, out, stream=None):
        ns = xi.shape[0]
        _check(lib().fmgmc_synthesize_field(self._h, level, ns, _ptr(xi), _ptr(out), _stream_ptr(stream)))
        return out

    def solve_level(self, level, xi, q_fine, q_coarse, cycles=None, flags=None, stream=None,
                    allow=(ENOTCONV, ENONFINITE)):
        """Returns the library's status code (OK / ENOTCONV / ENONFINITE); raises on others."""
        ns = xi.shape[0]
        rc = lib().fmgmc_solve_level(self._h, level, ns, _ptr(xi), _ptr(q_fine), _ptr(q_coarse),
                                     _ptr(cycles), _ptr(flags), _stream_ptr(stream))
        return _check(rc, allow)


    def solve_levels(self, xis, q_fines, q_coarses, cycles=None, flags=None, stream=None,
                     allow=(ENOTCONV, ENONFINITE)):
        """All levels at once (level l gets xis[l], ...); returns the status code."""
        L = len(xis)
        ns = np.array([int(x.shape[0]) for x in xis], np.int64)
        tabs = [(C.c_void_p * L)(*[_ptr(x) for x in xs]) if xs is not None else None
                for xs in (xis, q_fines, q_coarses, cycles, flags)]
        rc = lib().fmgmc_solve_levels(self._h, L, _ptr(ns),
                                      *[C.addressof(t) if t is not None else None for t in tabs],
                                      _stream_ptr(stream))
        return _check(rc, allow)

    def autotune(self, level, xi_pilot):
        """Measured schedule (check interval, graphs, batch) for a level."""
        p = np.zeros(3, np.int32)
        _check(lib().fmgmc_autotune(self._h, level, xi_pilot.shape[0], _ptr(xi_pilot), _ptr(p)))
        return dict(check_every=int(p[0]), graphs=int(p[1]), batch=int(p[2]))

    def set_schedule(self, level, check_every=1, graphs=0, batch=0):
        p = np.array([check_every, graphs, batch], np.int32)
        _check(lib().fmgmc_set_schedule(self._h, level, _ptr(p)))

    def schedule(self, level):
        p = np.zeros(3, np.int32)
        _check(lib().fmgmc_get_schedule(self._h, level, _ptr(p)))
        return dict(check_every=int(p[0]), graphs=int(p[1]), batch=int(p[2]))


    def set_warm_start(self, cnn, min_n=256, max_n=0):
        """Warm-start QoI stages with min_n <= n <= max_n (0: no bound) from `cnn` (None: off)."""
        self._warm = cnn  # keep the network alive while the context uses it
        _check(lib().fmgmc_set_warm_range(self._h, cnn._h if cnn is not None else None, min_n, max_n))

    def make_data(self, level, xi, x_coarse, t_coarse, x_fine, t_fine, stream=None):
        """Training pairs of the two QoI stages (device float32 buffers)."""
        return _check(lib().fmgmc_cnn_make_data(self._h, level, xi.shape[0], _ptr(xi), _ptr(x_coarse),
                                                _ptr(t_coarse), _ptr(x_fine), _ptr(t_fine), _stream_ptr(stream)),
                      (ENOTCONV,))

    def train_cnn(self, cnn, level, xi, batch, lr):
        """Native training loop; returns the loss after every Adam step."""
        n = xi.shape[0]
        steps = -(-n // min(batch, n))
        hist = np.full(steps * (2 if level >= 1 else 1), np.nan)
        _check(lib().fmgmc_cnn_train(self._h, cnn._h, level, n, _ptr(xi), batch, lr, _ptr(hist)))
        return hist[np.isfinite(hist)]


class Cnn:
    """The warm-start network (2 -> 32 -> 4 residual 32 -> 1, 3x3)."""
    NPARAMS = 37889

    def __init__(self, seed=0, device=0, path=None):
        h = _VP()
        _check(lib().fmgmc_cnn_create(C.byref(h), seed, device))
        self._h = h
        if path is not None:
            self.load(path)

    def close(self):
        if getattr(self, "_h", None):
            lib().fmgmc_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self):
        out = np.zeros(self.NPARAMS, np.float32)
        _check(lib().fmgmc_cnn_get_params(self._h, _ptr(out)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32) if isinstance(theta, np.ndarray) else theta
        _check(lib().fmgmc_cnn_set_params(self._h, _ptr(theta)))

    def save(self, path):
        _check(lib().fmgmc_cnn_save(self._h, os.fsencode(path)))

    def load(self, path):
        _check(lib().fmgmc_cnn_load(self._h, os.fsencode(path)))

    def forward(self, x, y, prec="bf16", stream=None):
        """x [B][2][n][n], y [B][n][n]: device float32 tensors."""
        _check(lib().fmgmc_cnn_forward(self._h, x.shape[-1], x.shape[0], _ptr(x), _ptr(y),
                                       CNN_PREC[prec], _stream_ptr(stream)))
        return y

    def grad(self, x, t=None, grad=None, loss="error", stream=None):
        """Loss ("error" against targets t, or "residual") and gradient into `grad` if given."""
        val = C.c_double()
        _check(lib().fmgmc_cnn_grad(self._h, x.shape[-1], x.shape[0], _ptr(x), _ptr(t), CNN_LOSS[loss],
                                    C.byref(val), _ptr(grad), _stream_ptr(stream)))
        return val.value

    def adam(self, lr, stream=None):
        _check(lib().fmgmc_cnn_adam(self._h, lr, _stream_ptr(stream)))


CNN_PREC = {"fp32": 0, "bf16": 1, "bf16_fused": 2}
CNN_LOSS = {"error": 0, "residual": 1}


def _check_count(rc):
    if rc < 0:
        raise FmgmcError(rc, last_error())
    return rc


def _level_dict(o):
    return dict(n=o.n, mean_y=o.mean_y, var_y=o.var_y, mean_qf=o.mean_qf, var_qf=o.var_qf, mean_qc=o.mean_qc)


def estimate(qf_levels, qc_levels, n_shifts=1, stream=None):
    """MLMC / MLQMC estimate over levels; arrays host or device (float64, 1-D).
    Without a stream (and at most MAX_LEVELS levels) through fmgmc_estimate, the
    aggregate form; with one through fmgmc_estimate_levels on that stream."""
    L = len(qf_levels)
    n = np.array([int(q.shape[0]) for q in qf_levels], np.int64)
    pf = (C.c_void_p * L)(*[_ptr(q) for q in qf_levels])
    pc = (C.c_void_p * L)(*[_ptr(q) for q in qc_levels])
    if stream is None and L <= MAX_LEVELS:
        e = Est()
        _check(lib().fmgmc_estimate(L, _ptr(n), C.cast(pf, C.c_void_p), C.cast(pc, C.c_void_p), n_shifts,
                                    C.byref(e)))
        return dict(levels=[_level_dict(e.level[l]) for l in range(e.n_levels)], mean=e.mean,
                    var_of_mean=e.var_of_mean)
    out = (LevelEst * L)()
    mean = C.c_double()
    var = C.c_double()
    _check(lib().fmgmc_estimate_levels(L, _ptr(n), C.cast(pf, C.c_void_p), C.cast(pc, C.c_void_p), n_shifts,
                                       C.cast(out, C.c_void_p), C.byref(mean), C.byref(var),
                                       _stream_ptr(stream)))
    return dict(levels=[_level_dict(o) for o in out], mean=mean.value, var_of_mean=var.value)


def estimate_noalloc(qf_levels, qc_levels, n_shifts=1, stream=None):
    """The estimate of estimate(), through the entry point that allocates nothing
    (device arrays only; n_shifts <= 4096)."""
    L = len(qf_levels)
    n = np.array([int(q.shape[0]) for q in qf_levels], np.int64)
    pf = (C.c_void_p * L)(*[_ptr(q) for q in qf_levels])
    pc = (C.c_void_p * L)(*[_ptr(q) for q in qc_levels])
    out = (LevelEst * L)()
    mean = C.c_double()
    var = C.c_double()
    _check(lib().fmgmc_estimate_levels_noalloc(L, _ptr(n), C.cast(pf, C.c_void_p), C.cast(pc, C.c_void_p),
                                               n_shifts, C.cast(out, C.c_void_p), C.byref(mean), C.byref(var),
                                               _stream_ptr(stream)))
    return dict(levels=[_level_dict(o) for o in out], mean=mean.value, var_of_mean=var.value)


def header_functions():
    """Names of the functions declared in include/fmgmc.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "fmgmc.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(fmgmc_\w+)\s*\(", txt, re.M)))
