"""C ABI of the HIP library: loads, exports every declared symbol, host-side logic.

Runs without a GPU: no call here launches device work.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1910_04727_amd import fmgmc


def test_library_exports_every_header_function():
    L = fmgmc.lib()
    names = fmgmc.header_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(L, name), name
    assert L.fmgmc_version() >= 100


@pytest.mark.parametrize("sigma2,corr_len,M", [(1.0, 0.3, 64), (1.0, 0.2, 256), (2.0, 0.1, 512),
                                               (3.0, 0.05, 1024)])
def test_mode_table_equals_oracle(sigma2, corr_len, M):
    a, b, lam = fmgmc.kl_modes(sigma2, corr_len, M)
    oa, ob, olam = O.kl_table(sigma2, corr_len, M)
    assert np.array_equal(a, oa) and np.array_equal(b, ob)
    assert np.max(np.abs(lam - olam) / olam) < 1e-13


def test_mode_table_rejects_bad_field():
    z = np.zeros(4, np.int32)
    lam = np.zeros(4)
    L = fmgmc.lib()
    assert L.fmgmc_kl_modes(1.0, -0.1, 4, z.ctypes.data, z.ctypes.data, lam.ctypes.data) == fmgmc.EINVAL
    assert L.fmgmc_kl_modes(0.0, 0.1, 4, z.ctypes.data, z.ctypes.data, lam.ctypes.data) == fmgmc.EINVAL
    assert L.fmgmc_kl_modes(1.0, 0.1, 0, z.ctypes.data, z.ctypes.data, lam.ctypes.data) == fmgmc.EINVAL
    assert "invalid" in fmgmc.last_error()


@pytest.mark.parametrize("bad", [
    dict(n0=12),                 # not a power of two
    dict(n0=2),                  # below the coarsest grid
    dict(n_levels=0),
    dict(n0=1024, n_levels=2),   # finest grid above 1024
    dict(solver="fp32_ir", n0=4),
    dict(nu1=3),
    dict(rel_tol=0.0),
])
def test_create_validates_before_touching_a_device(bad):
    kw = dict(sigma2=1.0, corr_len=0.3, n_modes=64, n_levels=3, n0=16)
    kw.update(bad)
    with pytest.raises(fmgmc.FmgmcError) as e:
        fmgmc.Context(**kw)
    assert e.value.code == fmgmc.EINVAL


def test_estimate_rejects_bad_sizes():
    with pytest.raises(fmgmc.FmgmcError):
        fmgmc.estimate([np.zeros(10)], [np.zeros(10)], n_shifts=3)


def test_flag_bits_follow_the_boundary_contract():
    """bit 0 not converged, bit 1 non-finite, bit 2 re-solved by the FP64 form;
    the rejected learned start is an extra bit above them."""
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(fmgmc.HERE), "include", "fmgmc.h")).read()
    vals = dict((k, int(v)) for k, v in re.findall(r"FMGMC_FLAG_(\w+)\s*=\s*(\d+)", hdr))
    assert vals == {"NOTCONV": 1, "NONFINITE": 2, "FP64": 4, "WARM_REJECTED": 8}
    assert (fmgmc.FLAG_NOTCONV, fmgmc.FLAG_NONFINITE, fmgmc.FLAG_FP64, fmgmc.FLAG_WARM_REJECTED) == (1, 2, 4, 8)


def test_binding_structs_match_the_c_header(tmp_path):
    """The ctypes structs of the binding have the header's sizes and field offsets
    (a plain C program compiled against include/fmgmc.h prints them)."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(fmgmc.HERE), "include")
    structs = {"fmgmc_field": fmgmc.Field, "fmgmc_hier": fmgmc.Hier, "fmgmc_opts": fmgmc.Opts,
               "fmgmc_level_est": fmgmc.LevelEst, "fmgmc_est": fmgmc.Est}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmgmc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", inc, str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)]).decode().splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("bad", [
    dict(cnn_weights="w.bin"),                      # warm start needs the FP32_IR solver
    dict(solver="fp32_ir", cnn_weights="w.bin", case=1),   # and Case II
    dict(solver="fp32_ir", cnn_weights="w.bin", warm_min_n=8),
])
def test_create_validates_warm_start_options(bad):
    kw = dict(sigma2=1.0, corr_len=0.3, n_modes=64, n_levels=3, n0=16)
    kw.update(bad)
    with pytest.raises(fmgmc.FmgmcError) as e:
        fmgmc.Context(**kw)
    assert e.value.code == fmgmc.EINVAL


def test_aggregate_estimate_rejects_too_many_levels():
    L = 17
    n = np.full(L, 4, np.int64)
    q = [np.zeros(4) for _ in range(L)]
    pf = (C.c_void_p * L)(*[a.ctypes.data for a in q])
    out = fmgmc.Est()
    rc = fmgmc.lib().fmgmc_estimate(L, n.ctypes.data, C.cast(pf, C.c_void_p), C.cast(pf, C.c_void_p), 1,
                                    C.byref(out))
    assert rc == fmgmc.EINVAL and "FMGMC_MAX_LEVELS" in fmgmc.last_error()
