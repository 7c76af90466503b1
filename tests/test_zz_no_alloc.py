"""The allocation-free estimator entry point against the allocating one.

fmgmc_estimate_levels_noalloc runs the same reduction kernel as
fmgmc_estimate_levels in the library's fixed device scratch, so its results
must be the same bits. Two calls in a row, the second on smaller inputs,
check that nothing of the first call's larger contents leaks into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fmgmc.lib()


def log(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def same(a, b):
    assert a["mean"] == b["mean"] and a["var_of_mean"] == b["var_of_mean"]
    for x, y in zip(a["levels"], b["levels"]):
        for k in ("n", "mean_y", "var_y", "mean_qf", "var_qf", "mean_qc"):
            assert x[k] == y[k], k


def levels(rng, sizes, scale=1.0):
    out = []
    for n in sizes:
        qf = rng.standard_normal(n) * scale + 1.0
        qc = 0.3 * rng.standard_normal(n)
        out.append((dev(qf), dev(qc), qf, qc))
    return out


def test_noalloc_monte_carlo_two_calls():
    rng = np.random.default_rng(2024)
    for call, sizes in enumerate([(100000, 20011, 4096), (513, 7)]):
        lv = levels(rng, sizes)
        log(f"noalloc MC call {call + 1}: sizes {sizes}")
        ref = fmgmc.estimate([a for a, _, _, _ in lv], [b for _, b, _, _ in lv], stream=torch.cuda.current_stream())
        got = fmgmc.estimate_noalloc([a for a, _, _, _ in lv], [b for _, b, _, _ in lv])
        same(got, ref)
        # and the oracle's statistics of the same numbers (to rounding)
        for l, (_, _, qf, qc) in enumerate(lv):
            s = O.level_stats(qf, qc)
            assert abs(got["levels"][l]["mean_y"] - s["mean_y"]) <= 1e-13 * max(1.0, abs(s["mean_y"]))
            assert abs(got["levels"][l]["var_y"] - s["var_y"]) <= 1e-12 * max(1.0, abs(s["var_y"]))


def test_noalloc_rqmc_two_calls():
    rng = np.random.default_rng(99)
    for call, (R, npts) in enumerate([(64, 2048), (16, 32)]):
        qf = rng.standard_normal(R * npts)
        qc = 0.5 * rng.standard_normal(R * npts)
        log(f"noalloc RQMC call {call + 1}: {R} shifts x {npts} points")
        ref = fmgmc.estimate([dev(qf)], [dev(qc)], n_shifts=R, stream=torch.cuda.current_stream())
        got = fmgmc.estimate_noalloc([dev(qf)], [dev(qc)], n_shifts=R)
        same(got, ref)
        s = O.rqmc_stats(qf, qc, R)
        assert abs(got["levels"][0]["mean_y"] - s["mean_y"]) < 1e-14
        assert abs(got["levels"][0]["var_y"] / s["var_mean"] - 1) < 1e-12


def test_noalloc_rejects_what_it_cannot_do_without_allocating():
    a = np.zeros(64)
    with pytest.raises(fmgmc.FmgmcError) as e:
        fmgmc.estimate_noalloc([a], [a])           # host arrays need a staging buffer
    assert e.value.code == fmgmc.EINVAL
    d = dev(np.zeros(4097 * 2))
    with pytest.raises(fmgmc.FmgmcError) as e:
        fmgmc.estimate_noalloc([d], [d], n_shifts=4097)   # beyond the scratch's shift slots
    assert e.value.code == fmgmc.EINVAL and "4096" in fmgmc.last_error()
