"""Freezes the per-level sample counts of the 5-level Darcy configuration.

Configuration: fine grids 32^2 .. 512^2, sigma^2 = 1, correlation length 0.2,
256 KL modes. A pilot of 256 samples per level (pilot seed stream) is solved
by the CPU oracle; V_l is the sample variance of Y_l = Q^f_l - Q^c_l and C_l
the oracle's measured seconds per sample. The optimal counts for RMSE 1e-3
(Section 2.1, Lagrange-multiplier allocation) are then scaled so that the
finest level gets 4096 samples, rounded up. Output: cfg2_nl.json beside this
script. Calls only the oracle; run from the repository root:

    python tests/golden/make_cfg2_nl.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1910_04727_amd import inputs  # noqa: E402

SIGMA2, CORR, M, N_LEVELS, N0 = 1.0, 0.2, 256, 5, 32
PILOT, EPS, N_FINEST = 256, 1e-3, 4096


def main():
    tab = O.kl_table(SIGMA2, CORR, M)
    V, C = [], []
    for l in range(N_LEVELS):
        xi = inputs.mc_normals(PILOT, M, config=2, level=l, purpose=inputs.PURPOSE_PILOT)
        t0 = time.perf_counter()
        qf, qc, _, fl = O.solve_level(SIGMA2, CORR, tab, N0 << l, l, xi, nthreads=O.max_threads())
        dt = time.perf_counter() - t0
        assert not fl.any()
        V.append(O.level_stats(qf, qc)["var_y"])
        C.append(dt / PILOT)
        print(f"level {l}: n {N0 << l} V {V[-1]:.4e} C {C[-1]:.3e} s/sample", flush=True)
    n_opt = O.optimal_nl(V, C, EPS)
    scale = N_FINEST / n_opt[-1]
    n_l = [int(np.ceil(x * scale)) for x in n_opt]
    n_l[-1] = N_FINEST
    out = dict(levels=[N0 << l for l in range(N_LEVELS)], pilot=PILOT, eps=EPS, V=V, C_seconds=C,
               n_opt=[int(x) for x in n_opt], n_l=n_l, threads=O.max_threads())
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_nl.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["n_l"])


if __name__ == "__main__":
    main()
