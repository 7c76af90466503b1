"""Adaptive drivers on the library against the same drivers on the oracle:
identical sample sets, so identical decisions (levels, sample counts) and
estimates equal to the solver's accuracy."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import drivers, fmgmc

pytestmark = pytest.mark.gpu

CFG = dict(sigma2=1.0, corr_len=0.3, n_modes=16, n_levels=3, n0=16)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def oracle_solver():
    tab = O.kl_table(CFG["sigma2"], CFG["corr_len"], CFG["n_modes"])

    def solve(jobs):
        return {l: O.solve_level(CFG["sigma2"], CFG["corr_len"], tab, CFG["n0"] << l, l, xi,
                                 nthreads=O.max_threads())[:2] for l, xi in jobs.items()}
    return solve


@pytest.mark.parametrize("kind", ["mlmc", "mlqmc", "mlqmc_lattice"])
def test_driver_on_library_equals_driver_on_oracle(kind):
    if kind == "mlmc":
        run = lambda s: drivers.mlmc(s, 1e-2, M=16, config=9, levels_available=3, n_init=32)
    else:
        rule = "lattice" if kind == "mlqmc_lattice" else "sobol"
        run = lambda s: drivers.mlqmc(s, 4e-3, M=16, config=9, levels_available=3, m_init=4, nshift=8, rule=rule)
    with fmgmc.Context(**CFG) as ctx:
        rg = run(drivers.library_solver(ctx))
    ro = run(oracle_solver())
    print(f"{kind}: L {rg.L} N {rg.N} mean {rg.mean:.12f} (oracle {ro.mean:.12f})", flush=True)
    assert rg.L == ro.L and rg.N == ro.N
    assert abs(rg.mean - ro.mean) <= 1e-9 * abs(ro.mean)
    assert rg.var_of_mean <= (1e-2 if kind == "mlmc" else 4e-3) ** 2 / 2 * (1 + 1e-12)
