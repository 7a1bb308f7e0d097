"""The C-ABI library loads and exports every symbol include/mbl.h declares;
host-only entry points agree with the oracle (no GPU needed)."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1411_0660_amd as mbl
from conftest import ROOT


def _declared():
    txt = open(os.path.join(ROOT, "include", "mbl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mbl_[a-z_0-9]+)\s*\(", txt)))


def test_header_matches_binding_list():
    assert sorted(mbl.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = mbl.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mbl.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (mbl_\w+)", out))
    assert set(_declared()) <= exported


def test_library_is_gfx950_code_object():
    data = open(mbl.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_sector_dim_and_errors():
    assert mbl.mbl_sector_dim(22) == 705432
    assert mbl.mbl_sector_dim(20) == 184756
    assert mbl.mbl_sector_dim(19) == 92378 and mbl.mbl_sector_dim(3) == 3   # S^z = +1/2
    assert mbl.mbl_sector_dim(1) == -1 and mbl.mbl_sector_dim(24) == -1
    assert mbl.lib().mbl_strerror(mbl.MBL_EINVAL) == b"invalid argument"


def test_fields_match_oracle_generator():
    for L, h, seed in [(12, 3.0, 0), (20, 2.0, 4), (18, 5.0, 123456789)]:
        a = mbl.mbl_fields(L, h, seed)
        b = oracle.fields(L, h, seed)
        assert np.array_equal(a, b)


def test_problem_init_defaults():
    p = mbl.mbl_problem()
    mbl.lib().mbl_problem_init(ctypes.byref(p))
    assert p.J == 1.0 and math.isnan(p.sigma) and p.prec == mbl.MBL_FP64
    assert p.flags & mbl.MBL_WANT_OBS


def test_disorder_average_matches_oracle():
    # host arithmetic of the library (no device work) against the oracle's
    rng = np.random.default_rng(5)
    B = rng.normal(size=(7, mbl.MBL_NBIN))
    B[:, 4] = B[:, 3] ** 2 + rng.uniform(0.1, 1.0, size=7)
    B[2, 0] = math.nan
    B[5, 7] = math.inf
    got = mbl.mbl_disorder_average(B)
    ref = oracle.disorder_average(B)
    assert np.allclose(got["mean"], ref["mean"], rtol=1e-14, atol=0, equal_nan=True)
    assert np.allclose(got["sem"], ref["sem"], rtol=1e-13, atol=0, equal_nan=True)
    assert got["sigma_e"] == pytest.approx(ref["sigma_e"], rel=1e-13)
    with pytest.raises(mbl.MblError):
        mbl.mbl_disorder_average(np.zeros((0, mbl.MBL_NBIN)))


def test_struct_layouts_match_header(tmp_path):
    # every ctypes structure of the binding has the size and field offsets the
    # C compiler gives the header's struct (a drifted binding reads shifted fields)
    structs = [mbl.mbl_problem, mbl.mbl_result, mbl.mbl_symbolic_info, mbl.mbl_kernel_profile,
               mbl.mbl_serve_info, mbl.mbl_solve_info]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mbl.h"', 'int main(void) {']
    for S in structs:
        n = S.__name__
        lines.append(f'printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in S._fields_:
            lines.append(f'printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    want = []
    for S in structs:
        n = S.__name__
        want.append(f"{n} size {ctypes.sizeof(S)}")
        want += [f"{n} {f} {getattr(S, f).offset}" for f, _ in S._fields_]
    assert [g for g in got if g] == want
