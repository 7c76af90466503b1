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
  - Randomly shifted rank-1 lattice rules (Section 2.4), as an embedded
    (extensible) lattice sequence in base 2: point i of the sequence is
    {phi_2(i) z + Delta}, phi_2 the radical inverse, so the first 2^m points
    are the 2^m-point lattice rule {k z / 2^m} for every m. The generating
    vector z (odd integers below 2^m_max) is chosen component by component
    (Sloan and Reztsov 2002; the fast FFT form over the unit group of
    Z_(2^m), after Nuyens and Cools 2006 and Cools, Kuo and Nuyens 2006) from
    the shift-averaged worst-case error of the weighted unanchored Sobolev
    space with product weights gamma_j = j^-2,
      e^2_n(z) = -1 + (1/n) sum_{k<n} prod_j (1 + gamma_j B2({k z_j / n})),
      B2(x) = x^2 - x + 1/6;
    in each dimension the candidate minimising max_m e^2_(2^m) / min e^2_(2^m)
    over m_min <= m <= m_max is kept. Shifts are 30-bit integers as for
    Sobol' below, with the same cell-midpoint mapping.
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


def _b2(x):
    return x * x - x + 1.0 / 6.0


def _pow5_table(q):
    """5^b mod 2^q for b = 0 .. 2^(q-2) - 1 (with -1 these generate the odd residues)."""
    cnt = 1 << (q - 2)
    out = np.empty(cnt, dtype=np.int64)
    v, mod = 1, 1 << q
    for b in range(cnt):
        out[b] = v
        v = v * 5 % mod
    return out


def lattice_cbc(m_max, gammas, m_min=4, table=False):
    """Generating vector of an embedded base-2 lattice sequence by fast CBC.

    Returns z (int64, one odd entry per weight). Candidates are z = 5^a mod
    2^m_max, a < 2^(m_max-2); -z gives the same errors (B2 is symmetric), and
    e^2_(2^q) depends on a only modulo 2^(q-2). With table=True also returns,
    per dimension, the list over q = m_min .. m_max of e^2_(2^q) for
    a = 0 .. 2^(q-2) - 1, given the previous components."""
    m = int(m_max)
    if not (3 <= m_min <= m <= 30):
        raise ValueError("need 3 <= m_min <= m_max <= 30")
    n = 1 << m
    gammas = np.asarray(gammas, float)
    k = np.arange(n, dtype=np.int64)
    P = np.ones(n)
    # level q holds the points k = 2^(m-q) u, u odd below 2^q; u = +-5^b mod 2^q
    reps = {q: _pow5_table(q) for q in range(3, m + 1)}
    fw = {q: np.fft.rfft(_b2(reps[q] / float(1 << q))) for q in reps}
    z, tabs = [], []
    for gj in gammas:
        tot = np.array([P[0] * (1.0 + gj / 6.0)])   # sum over the points so far, per candidate class
        crit = None
        Es = []
        for q in range(1, m + 1):
            t = m - q
            if q <= 2:
                # one or two odd residues, with B2(u / 2^q) the same for all of them
                us = np.arange(1, 1 << q, 2, dtype=np.int64)
                tot = tot + np.sum(P[us << t]) * (1.0 + gj * _b2(1.0 / (1 << q)))
                continue
            r = reps[q]
            Pt = P[r << t] + P[((1 << q) - r) << t]
            L = r.size
            # corr[a] = sum_b Pt[b] B2({5^(a+b) / 2^q}), a cyclic correlation over the unit group
            corr = np.fft.irfft(np.conj(np.fft.rfft(Pt)) * fw[q], L)
            tot = np.tile(tot, L // tot.size) + np.sum(Pt) + gj * corr
            if q >= m_min:
                E = tot / float(1 << q) - 1.0
                ratio = E / E.min()
                crit = ratio if crit is None else np.maximum(np.tile(crit, L // crit.size), ratio)
                if table:
                    Es.append(E)
        a = int(np.argmin(crit))
        zj = int(reps[m][a])
        z.append(zj)
        if table:
            tabs.append(Es)
        P *= 1.0 + gj * _b2(((k * zj) & (n - 1)) / float(n))
    z = np.array(z, dtype=np.int64)
    return (z, tabs) if table else z


_LATTICE_CACHE = {}


def lattice_vector(M, m_max=16):
    """Generating vector for M dimensions with weights j^-2 (cached)."""
    key = (M, m_max)
    if key not in _LATTICE_CACHE:
        _LATTICE_CACHE[key] = lattice_cbc(m_max, 1.0 / np.arange(1, M + 1, dtype=float) ** 2)
    return _LATTICE_CACHE[key]


def _bitrev(i, m):
    i = np.asarray(i, dtype=np.int64)
    r = np.zeros_like(i)
    for b in range(m):
        r |= ((i >> b) & 1) << (m - 1 - b)
    return r


def lattice_ints(M, m_from, m_to, m_max=16):
    """Points 2^m_from .. 2^m_to - 1 of the lattice sequence (all from 0 if
    m_from < 0) as exact 30-bit integers: [count, M] uint64 of
    (phi_2(i) z mod 1) * 2^30."""
    if m_to > m_max:
        raise ValueError("m_to beyond the generating vector's m_max")
    z = lattice_vector(M, m_max) & ((1 << m_to) - 1)
    lo = 0 if m_from < 0 else (1 << m_from)
    kk = _bitrev(np.arange(lo, 1 << m_to, dtype=np.int64), m_to)
    pts = (kk[:, None] * z[None, :]) & ((1 << m_to) - 1)
    return (pts << (_BITS - m_to)).astype(np.uint64)


def _lattice_shifts(M, nshift, config, level, seed):
    ss = np.random.SeedSequence([seed, config, level, 9])
    g = np.random.Generator(np.random.PCG64(ss))
    return g.integers(0, 1 << _BITS, size=(nshift, M), dtype=np.uint64)


def lattice_normals_range(M, m_from, m_to, nshift, config, level, seed=SEED, m_max=16):
    """Randomly shifted lattice points 2^m_from .. 2^m_to - 1: [nshift, count, M]
    normals, u = ((x + Delta_r) mod 2^30 + 1/2) 2^-30 through the inverse
    normal CDF."""
    from scipy.special import ndtri
    base = lattice_ints(M, m_from, m_to, m_max)
    sh = _lattice_shifts(M, nshift, config, level, seed)
    out = np.empty((nshift, base.shape[0], M))
    mask = np.uint64((1 << _BITS) - 1)
    for r in range(nshift):
        kk = (base + sh[r][None, :]) & mask
        out[r] = ndtri((kk.astype(np.float64) + 0.5) * (1.0 / float(1 << _BITS)))
    return out
