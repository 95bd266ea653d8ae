"""The C-ABI library loads and exports every symbol include/*.h declares, and
rejects invalid input with documented status codes before touching the GPU.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1704_07458_amd import binding as B
from paper_1704_07458_amd import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[\w\s\*]+?\b(lobpcg_\w+)\s*\(", text, flags=re.M):
            if "typedef" in text[max(0, m.start() - 40):m.start() + 10]:
                continue
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    # the binding describes exactly the declared set
    assert set(declared) == set(B.SIGNATURES)


def test_default_options_values():
    o = B.default_options()
    assert o.maxit == 2000 and o.precision == 0 and o.tau_ortho == 1e-12
    assert o.drop_factor == 10.0 and o.skip_factor == 10.0 and o.implicit_products == -1
    assert o.ortho_mode == 0 and o.force_ortho == 0 and o.implicit_gram == 1 and o.largest == 0
    assert o.basic == 0


def _create(A, k, B_=None, **kw):
    lib = B.load()
    keep = []
    a = B._csr_struct(A, keep)
    b = B._csr_struct(B_, keep) if B_ is not None else None
    o = B.default_options()
    for key, val in kw.items():
        setattr(o, key, val)
    h = C.c_void_p()
    code = lib.lobpcg_create(C.byref(h), C.byref(a), C.byref(b) if b is not None else None, k,
                             C.byref(o))
    if code == 0:
        lib.lobpcg_destroy(h)
    return code, lib.lobpcg_last_error().decode()


def test_rejects_unsorted_columns():
    A = P.laplacian_2d_dirichlet(8)
    A.colind = A.colind.copy()
    r = 5
    s, e = A.rowptr[r], A.rowptr[r + 1]
    A.colind[s:e] = A.colind[s:e][::-1]
    code, msg = _create(A, 2)
    assert code == -1 and "sorted" in msg


def test_rejects_bad_rowptr_and_column_range():
    A = P.laplacian_2d_dirichlet(8)
    A.rowptr = A.rowptr.copy()
    A.rowptr[-1] += 1
    code, msg = _create(A, 2)
    assert code == -1
    A = P.laplacian_2d_dirichlet(8)
    A.colind = A.colind.copy()
    A.colind[3] = 10_000
    code, msg = _create(A, 2)
    assert code == -1 and "range" in msg


def test_rejects_block_too_wide_and_bad_k():
    A = P.laplacian_2d_dirichlet(4)  # n = 16
    code, msg = _create(A, 6)  # n_x = 7, 3 n_x = 21 > 16
    assert code == -1 and "3 * block_size" in msg
    code, _ = _create(A, 0)
    assert code == -1
    code, _ = _create(A, 3, block_size=2)
    assert code == -1


def test_rejects_implicit_products_with_B_and_bad_ortho_mode():
    A = P.laplacian_2d_dirichlet(8)
    Bm = P.laplacian_2d_dirichlet(8)
    code, msg = _create(A, 2, Bm, implicit_products=1)
    assert code == -1 and "B = I" in msg
    code, msg = _create(A, 2, implicit_products=2)
    assert code == -1 and "implicit_products" in msg
    code, msg = _create(A, 2, ortho_mode=2)
    assert code == -1 and "ortho_mode" in msg
    code, msg = _create(A, 2, largest=2)
    assert code == -1 and "largest" in msg
    code, msg = _create(A, 2, basic=2)
    assert code == -1 and "basic" in msg


def test_rejects_mismatched_B_and_nonfinite_values():
    A = P.laplacian_2d_dirichlet(8)
    Bm = P.laplacian_2d_dirichlet(6)
    code, msg = _create(A, 2, Bm)
    assert code == -1 and "mismatch" in msg
    A.values = A.values.copy()
    A.values[0] = np.nan
    code, msg = _create(A, 2)
    assert code == -1 and "non-finite" in msg


def test_null_handle_calls_fail_cleanly():
    lib = B.load()
    assert lib.lobpcg_solve(None, 1e-8, None, 0, B.PRECOND_FN(), None, None) == -1
    assert lib.lobpcg_eigpairs(None, 1, None, None, 1, None, 0) == -1
    lib.lobpcg_destroy(None)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the header's field names, offsets and size.

    A C program compiled against include/lobpcg.h prints offsetof for each field the
    binding declares and sizeof for each structure; a field added to one side only, or
    in a different order, changes an offset or the size.
    """
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [B.lobpcg_csr, B.lobpcg_zcsr, B.lobpcg_options, B.lobpcg_info,
               B.lobpcg_kernel_stat]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lobpcg.h"', "int main(void) {"]
    for S in structs:
        n = S.__name__
        lines.append(f'  printf("{n} sizeof %zu\\n", sizeof({n}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out.splitlines())}
    for S in structs:
        n = S.__name__
        assert got[(n, "sizeof")] == C.sizeof(S), n
        for f, _ in S._fields_:
            assert got[(n, f)] == getattr(S, f).offset, (n, f)


def _create_hermitian(A, k, Bm=None, **opts):
    lib = B.load()
    o = B.default_options()
    for key, val in opts.items():
        setattr(o, key, val)
    keep: list = []
    a = B._zcsr_struct(A, keep)
    b = B._zcsr_struct(Bm, keep) if Bm is not None else None
    h = C.c_void_p()
    code = lib.lobpcg_create_hermitian(C.byref(h), C.byref(a),
                                       C.byref(b) if b is not None else None, k, C.byref(o))
    if code == 0:
        lib.lobpcg_destroy(h)
    return code, lib.lobpcg_last_error().decode()


def test_hermitian_create_rejects_bad_input_before_the_gpu():
    A = P.twisted_laplacian_3d(4)  # n = 64
    bad = P.ZCSR(A.n, A.rowptr.copy(), A.colind, A.values_re, A.values_im)
    bad.rowptr[-1] += 1
    code, msg = _create_hermitian(bad, 2)
    assert code == -1 and "rowptr" in msg
    uns = P.ZCSR(A.n, A.rowptr, A.colind.copy(), A.values_re, A.values_im)
    s, e = A.rowptr[5], A.rowptr[6]
    uns.colind[s:e] = uns.colind[s:e][::-1]
    code, msg = _create_hermitian(uns, 2)
    assert code == -1 and "sorted" in msg
    code, _ = _create_hermitian(A, 0)
    assert code == -1
    code, msg = _create_hermitian(A, 20)  # n_x = 22, 3 n_x = 66 > 64
    assert code == -1 and "3 * block_size" in msg
    Bm, _ = P.twisted_pencil_3d(3)
    code, msg = _create_hermitian(A, 2, Bm)
    assert code == -1 and "order" in msg


def test_hermitian_calls_reject_null_and_real_handles():
    lib = B.load()
    assert lib.lobpcg_solve_hermitian(None, 1e-8, None, None, 0, B.PRECOND_FN(), None,
                                      None) == -1
    assert lib.lobpcg_eigpairs_hermitian(None, 1, None, None, None, 1, None, 0) == -1
