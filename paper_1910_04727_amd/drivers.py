"""Adaptive multilevel drivers of the paper, on the host around the library's
batched level solves.

  - mlmc: the adaptive MLMC loop (Section 2.2, Algorithm 1), which with the
    library's FMG pass is the FMG-MLMC loop (Section 2.5, Algorithm 3): Q^c_l
    comes with Q^f_l from one FMG pass. Start with levels 0..2 and n_init
    samples each; after every round of new samples re-estimate V_l, set
    N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)) (Section 2.3, the
    cost-minimising split of the variance eps^2 / 2), evaluate the extra
    samples, and when none are needed test the weak error by Richardson
    extrapolation, |mean Y_L| / (2^alpha - 1) < eps / sqrt(2); add a level if
    it fails.
  - mlqmc: the MLQMC loop (Section 2.4, Algorithm 2) with randomised point
    sets, scrambled Sobol' with digital shifts or an embedded lattice sequence
    with random shifts: while sum_l Var[Yhat_l] > eps^2 / 2, double the point set of
    the level maximising Var[Yhat_l] / (N_l C_l); then the same weak-error test.

Every per-sample computation (field, FMG solve, Q) runs in the library; the
drivers only choose sample counts. The solver is passed in as a function
jobs -> results ({level: xi [n, M]} -> {level: (q_fine, q_coarse)}), so the
same driver can run on the library (`library_solver`) or on any other
implementation of the level solve.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import inputs

CHUNK = 1 << 18  # samples per level generated and solved at once


def library_solver(ctx):
    """Solver function on a fmgmc.Context: all requested levels in one solve_levels call."""
    def solve(jobs):
        xis = [np.ascontiguousarray(jobs.get(l, np.zeros((0, ctx.n_modes)))) for l in range(ctx.n_levels)]
        qf = [np.zeros(x.shape[0]) for x in xis]
        qc = [np.zeros(x.shape[0]) for x in xis]
        ctx.solve_levels(xis, qf, qc)
        return {l: (qf[l], qc[l]) for l in jobs}
    return solve


def _mean(y):
    return math.fsum(y) / len(y) if len(y) else 0.0


def _var(y):
    if len(y) < 2:
        return 0.0
    m = _mean(y)
    return math.fsum((np.asarray(y) - m) ** 2) / (len(y) - 1)


def _rate(vals):
    """-slope of log2 |vals| against the level index over levels >= 1 (None if < 2 points)."""
    pts = [(l, math.log2(abs(v))) for l, v in enumerate(vals) if l >= 1 and v != 0 and np.isfinite(v)]
    if len(pts) < 2:
        return None
    x = np.array([p[0] for p in pts], float)
    y = np.array([p[1] for p in pts], float)
    return float(-np.polyfit(x, y, 1)[0])


@dataclass
class Result:
    mean: float                  # sum_l Yhat_l
    var_of_mean: float           # sum_l V_l / N_l (MC) or sum_l Var[Yhat_l] (QMC)
    L: int
    N: list                      # samples per level
    means: list                  # Yhat_l
    V: list                      # V_l (MC) or Var[Yhat_l] (QMC)
    alpha: float
    beta: float
    gamma: float
    bias: float                  # Richardson estimate |Yhat_L| / (2^alpha - 1)
    converged: bool
    rounds: list = field(default_factory=list)


def _cost_model(L, gamma):
    return [2.0 ** (gamma * l) for l in range(L + 1)]


def mlmc(solve, eps, M, config, levels_available, n_init=64, L_init=2, alpha=None, gamma=2.0,
         purpose=inputs.PURPOSE_ESTIMATOR, seed=inputs.SEED, max_rounds=64):
    """Adaptive (FMG-)MLMC. C_l = 2^(gamma l) (O(n_l^2) multigrid work); alpha
    from the level means when not given (at least 0.5). Samples of level l are
    rows 0, 1, 2, ... of its blocked PCG64 stream, so a run extends, never
    replaces, the samples it has."""
    L = min(L_init, levels_available - 1)
    Y = [np.zeros(0) for _ in range(L + 1)]
    dN = [n_init] * (L + 1)
    rounds = []
    converged = False
    for _ in range(max_rounds):
        # evaluate the extra samples of every level that needs them, in chunks
        while any(d > 0 for d in dN):
            jobs = {}
            for l, d in enumerate(dN):
                if d > 0:
                    take = min(d, CHUNK)
                    jobs[l] = inputs.mc_normals_blocked(len(Y[l]), take, M, config, l, purpose, seed)
                    dN[l] -= take
            res = solve(jobs)
            for l, (qf, qc) in res.items():
                Y[l] = np.concatenate([Y[l], np.asarray(qf) - np.asarray(qc)])
        N = [len(y) for y in Y]
        V = [_var(y) for y in Y]
        means = [_mean(y) for y in Y]
        C = _cost_model(L, gamma)
        s = sum(math.sqrt(v * c) for v, c in zip(V, C))
        Nopt = [math.ceil(2.0 / eps ** 2 * math.sqrt(v / c) * s) for v, c in zip(V, C)]
        dN = [max(0, no - n) for no, n in zip(Nopt, N)]
        a = alpha if alpha is not None else max(0.5, _rate(means) or 0.5)
        bias = abs(means[L]) / (2.0 ** a - 1.0)
        rounds.append(dict(L=L, N=N, Nopt=Nopt, V=V, means=means, alpha=a, bias=bias))
        if any(d > 0 for d in dN):
            continue
        if bias < eps / math.sqrt(2.0):
            converged = True
            break
        if L + 1 >= levels_available:
            break
        L += 1
        Y.append(np.zeros(0))
        dN.append(n_init)
    N = [len(y) for y in Y]
    V = [_var(y) for y in Y]
    means = [_mean(y) for y in Y]
    a = alpha if alpha is not None else max(0.5, _rate(means) or 0.5)
    return Result(mean=math.fsum(means), var_of_mean=math.fsum(v / n for v, n in zip(V, N)), L=L, N=N, means=means,
                  V=V, alpha=a, beta=_rate(V) or float("nan"), gamma=gamma,
                  bias=abs(means[L]) / (2.0 ** a - 1.0), converged=converged, rounds=rounds)


def mlqmc(solve, eps, M, config, levels_available, m_init=6, nshift=16, L_init=2, alpha=None, gamma=2.0,
          seed=inputs.SEED, max_rounds=200, m_max=None, rule="sobol"):
    """Adaptive MLQMC: level l holds nshift x 2^m_l samples (shift-major) of
    the randomised point set `rule` ("sobol" or "lattice"); Var[Yhat_l] is the
    variance of the mean over shifts. m_max defaults to 20 (Sobol') or 16
    (the lattice sequence's generating vector)."""
    if rule not in ("sobol", "lattice"):
        raise ValueError("rule must be 'sobol' or 'lattice'")
    if m_max is None:
        m_max = 20 if rule == "sobol" else 16
    if rule == "sobol":
        points = lambda l, m_from, m_to: inputs.rqmc_normals_range(M, m_from, m_to, nshift, config, l, seed)
    else:
        points = lambda l, m_from, m_to: inputs.lattice_normals_range(M, m_from, m_to, nshift, config, l, seed,
                                                                      m_max=m_max)
    L = min(L_init, levels_available - 1)
    m = [m_init] * (L + 1)
    Y = [None] * (L + 1)                  # per level: [nshift, 2^m_l]

    def extend(l, m_from, m_to):
        xi = points(l, m_from, m_to)  # [R, count, M]
        cnt = xi.shape[1]
        out = np.zeros((nshift, cnt))
        for r0 in range(0, nshift, max(1, CHUNK // max(cnt, 1))):
            r1 = min(nshift, r0 + max(1, CHUNK // max(cnt, 1)))
            qf, qc = solve({l: xi[r0:r1].reshape(-1, M)})[l]
            out[r0:r1] = (np.asarray(qf) - np.asarray(qc)).reshape(r1 - r0, cnt)
        Y[l] = out if Y[l] is None else np.concatenate([Y[l], out], axis=1)

    for l in range(L + 1):
        extend(l, -1, m[l])
    rounds = []
    converged = False
    for _ in range(max_rounds):
        shift_means = [np.array([_mean(Y[l][r]) for r in range(nshift)]) for l in range(L + 1)]
        means = [math.fsum(sm) / nshift for sm in shift_means]
        V = [math.fsum((sm - mu) ** 2) / (nshift * (nshift - 1)) for sm, mu in zip(shift_means, means)]
        C = _cost_model(L, gamma)
        N = [nshift << ml for ml in m]
        a = alpha if alpha is not None else max(0.5, _rate(means) or 0.5)
        bias = abs(means[L]) / (2.0 ** a - 1.0)
        rounds.append(dict(L=L, N=N, V=V, means=means, alpha=a, bias=bias))
        if math.fsum(V) > eps ** 2 / 2.0:
            l = int(np.argmax([v / (n * c) for v, n, c in zip(V, N, C)]))
            if m[l] >= m_max:
                break
            extend(l, m[l], m[l] + 1)
            m[l] += 1
            continue
        if bias < eps / math.sqrt(2.0):
            converged = True
            break
        if L + 1 >= levels_available:
            break
        L += 1
        m.append(m_init)
        Y.append(None)
        extend(L, -1, m_init)
    shift_means = [np.array([_mean(Y[l][r]) for r in range(nshift)]) for l in range(L + 1)]
    means = [math.fsum(sm) / nshift for sm in shift_means]
    V = [math.fsum((sm - mu) ** 2) / (nshift * (nshift - 1)) for sm, mu in zip(shift_means, means)]
    a = alpha if alpha is not None else max(0.5, _rate(means) or 0.5)
    return Result(mean=math.fsum(means), var_of_mean=math.fsum(V), L=L, N=[nshift << ml for ml in m], means=means,
                  V=V, alpha=a, beta=_rate(V) or float("nan"), gamma=gamma, bias=abs(means[L]) / (2.0 ** a - 1.0),
                  converged=converged, rounds=rounds)
