"""Seeded synthetic sample points (the random inputs of the method).

This module holds no arithmetic of the method itself: it only draws the
standard-normal KL coordinates xi that both the HIP library and the CPU
oracle consume, so that every form sees bit-identical inputs.

  - Monte Carlo (Section 2.1, Eq. (3)): i.i.d. N(0,1) from numpy's PCG64,
    seeded by SeedSequence([seed, config, level, purpose]); levels use
    independent streams, as the estimator requires (Eq. (5)).
  - Large Monte Carlo runs (millions of samples on a level) use a blocked
    variant: sample s of a level is row s % B of block s // B, each block an
    independent PCG64 stream seeded by SeedSequence([seed, config, level,
    purpose, block]), so blocks can be drawn in parallel and in any order.
  - Randomised QMC (Section 2.4): a scrambled Sobol' point set (scipy's
    Owen-type scrambling), then R random digital shifts (XOR of 30-bit
    integers), mapped through the inverse normal CDF at the dyadic cell
    midpoints u = (k + 1/2) 2^-30 so that u is never 0 or 1. Dimension m of
    the point set drives KL mode m (largest eigenvalue first). Samples are
    grouped shift-major: [shift][point][mode].
"""
import numpy as np

SEED = 20191010
PURPOSE_ESTIMATOR = 0
PURPOSE_PILOT = 1
PURPOSE_CNN_TRAIN = 2
PURPOSE_CNN_TEST = 3

_BITS = 30


def mc_normals(n, M, config, level, purpose=PURPOSE_ESTIMATOR, seed=SEED, offset=0):
    """[n, M] float64 standard normals for (config, level, purpose).

    `offset` skips that many leading rows of the same stream, so a batch can
    be regenerated in pieces with identical values.
    """
    ss = np.random.SeedSequence([seed, config, level, purpose])
    g = np.random.Generator(np.random.PCG64(ss))
    if offset:
        g.standard_normal((offset, M))
    return g.standard_normal((n, M))


MC_BLOCK = 65536


def _block_rows(config, level, purpose, seed, M, b, r0, r1):
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, config, level, purpose, b])))
    if r0:
        g.standard_normal((r0, M))
    return g.standard_normal((r1 - r0, M))


def mc_normals_blocked(start, n, M, config, level, purpose=PURPOSE_ESTIMATOR, seed=SEED, threads=16):
    """Rows [start, start + n) of the blocked stream, [n, M] float64."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((n, M))
    jobs = []
    s = start
    while s < start + n:
        b, r0 = divmod(s, MC_BLOCK)
        r1 = min(MC_BLOCK, r0 + (start + n - s))
        jobs.append((s - start, b, r0, r1))
        s += r1 - r0

    def run(j):
        o, b, r0, r1 = j
        out[o:o + r1 - r0] = _block_rows(config, level, purpose, seed, M, b, r0, r1)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(run, jobs))
    return out


def sobol_ints(M, m_log2, config, level, seed=SEED):
    """Scrambled Sobol' points as exact 30-bit integers, [2^m_log2, M] uint64."""
    from scipy.stats import qmc
    scr = int(np.random.SeedSequence([seed, config, level, 7]).generate_state(1)[0])
    s = qmc.Sobol(d=M, scramble=True, bits=_BITS, seed=scr)
    u = s.random_base2(m_log2)
    return np.round(u * float(1 << _BITS)).astype(np.uint64)


def _shifts(M, nshift, config, level, seed):
    ss = np.random.SeedSequence([seed, config, level, 8])
    g = np.random.Generator(np.random.PCG64(ss))
    return g.integers(0, 1 << _BITS, size=(nshift, M), dtype=np.uint64)


def _shifted_normals(base, shifts):
    from scipy.special import ndtri
    out = np.empty((shifts.shape[0], base.shape[0], base.shape[1]))
    for r in range(shifts.shape[0]):
        k = np.bitwise_xor(base, shifts[r][None, :])
        out[r] = ndtri((k.astype(np.float64) + 0.5) * (1.0 / float(1 << _BITS)))
    return out


def rqmc_normals(M, m_log2, nshift, config, level, seed=SEED):
    """[nshift * 2^m_log2, M] standard normals, grouped shift-major."""
    base = sobol_ints(M, m_log2, config, level, seed)
    return _shifted_normals(base, _shifts(M, nshift, config, level, seed)).reshape(nshift * base.shape[0], M)


def rqmc_normals_range(M, m_from, m_to, nshift, config, level, seed=SEED):
    """Points 2^m_from .. 2^m_to - 1 of the same scrambled Sobol' sequence and
    shifts as rqmc_normals (all points if m_from < 0): [nshift, count, M], so a
    point set can be doubled without recomputing the points it already has."""
    base = sobol_ints(M, m_to, config, level, seed)
    lo = 0 if m_from < 0 else (1 << m_from)
    return _shifted_normals(base[lo:], _shifts(M, nshift, config, level, seed))
