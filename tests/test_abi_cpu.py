"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/csvd.h declares, fills the paper's defaults, computes
the quadrature of Sec. 4 like the oracle does, and rejects malformed input
before touching the device."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import paper_2109_13655_amd as cs
from oracle import quadrature as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(csvd_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = cs.load()
    names = declared_functions()
    assert "csvd_solve_interval" in names and "csvd_probe_gather" in names and len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors of csvd_params and csvd_info have the size
    and the field offsets that the host C compiler gives the header's
    structs."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no host C compiler")
    structs = (cs.csvd_params, cs.csvd_info)
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "csvd.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.splitlines() if line)
    for st in structs:
        name = st.__name__
        assert int(got[f"{name} size"]) == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert int(got[f"{name}.{field}"]) == getattr(st, field).offset, (name, field)


def test_params_default_are_the_papers():
    p = cs.csvd_params_default()
    assert (p.L, p.M, p.N, p.ell) == (16, 8, 32, 1)
    assert p.delta == 1e-20 and p.alpha == 0.1
    assert p.transform == cs.CSVD_PLAIN and p.precision == cs.CSVD_FP64
    assert p.resid_target == 0.0 and p.ell_adaptive == 0


@pytest.mark.parametrize("transform", [cs.CSVD_PLAIN, cs.CSVD_EXP])
@pytest.mark.parametrize("N,M", [(16, 8), (32, 4), (2, 1)])
def test_quadrature_matches_oracle(transform, N, M):
    a, b = (0.4, 0.45) if transform == cs.CSVD_PLAIN else (1e-3, 1e-1)
    p = cs.csvd_params_default(N=N, M=M, transform=transform)
    shifts, w, c = cs.csvd_quadrature(a, b, p)
    sh_o, c_o = Q.moment_coeffs(a, b, N, M, 0.1, transform)
    np.testing.assert_allclose(shifts, sh_o, rtol=1e-14, atol=0)
    np.testing.assert_allclose(c, c_o, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(w, c_o[:, 0], rtol=1e-14)


def test_quadrature_rejects_bad_input():
    p = cs.csvd_params_default(N=15)
    with pytest.raises(cs.CsvdError):
        cs.csvd_quadrature(0.1, 0.2, p)
    p = cs.csvd_params_default(transform=cs.CSVD_EXP)
    with pytest.raises(cs.CsvdError):
        cs.csvd_quadrature(0.0, 0.2, p)
    p = cs.csvd_params_default()
    with pytest.raises(cs.CsvdError):
        cs.csvd_quadrature(0.3, 0.2, p)


def _csr_small():
    rp = np.array([0, 2, 3, 5, 6], dtype=np.int32)
    ci = np.array([0, 2, 1, 0, 2, 1], dtype=np.int32)
    va = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    return rp, ci, va


@pytest.mark.parametrize("case", ["m_lt_n", "bad_rowptr", "unsorted", "out_of_range", "nan", "rowptr_past_nnz"])
def test_create_rejects_malformed_csr(case):
    rp, ci, va = _csr_small()
    m, n = 4, 3
    code = cs.CSVD_EINVAL
    if case == "m_lt_n":
        m, n = 2, 3
        rp = rp[:3].copy()
    elif case == "bad_rowptr":
        rp = rp.copy(); rp[2] = 1
    elif case == "unsorted":
        ci = ci.copy(); ci[0], ci[1] = 2, 0
    elif case == "out_of_range":
        ci = ci.copy(); ci[2] = 3
    elif case == "nan":
        va = va.copy(); va[3] = np.nan
        code = cs.CSVD_ENUMERIC
    elif case == "rowptr_past_nnz":
        # a row pointer beyond nnz with a valid last entry: rejected before
        # any column index or value is read (the arrays hold nnz entries)
        rp = rp.copy(); rp[1] = 100
    with pytest.raises(cs.CsvdError) as e:
        cs.csvd_create(m, n, rp, ci, va)
    assert e.value.code == code


def test_oracle_transpose_definition():
    import synth
    from oracle import sparse
    I = synth.random_sparse(50, 30, 4, config=70)
    rp, ci, va = sparse.transpose(I.m, I.n, I.rowptr, I.colidx, I.vals)
    At = np.zeros((I.n, I.m))
    for j in range(I.n):
        At[j, ci[rp[j]:rp[j + 1]]] = va[rp[j]:rp[j + 1]]
    assert np.array_equal(At, I.dense().T)


def test_binding_checks_array_sizes():
    """The binding refuses arrays whose sizes do not match m and nnz before
    calling the library (which reads m + 1 row pointers and nnz entries)."""
    rp, ci, va = _csr_small()
    with pytest.raises(ValueError):
        cs.csvd_create(5, 3, rp, ci, va)          # rowptr needs m + 1 entries
    with pytest.raises(ValueError):
        cs.csvd_create(4, 3, rp, ci[:-1], va)     # colidx and vals differ in length
