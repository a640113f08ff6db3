"""C-ABI checks that need no GPU: the library loads, exports every function
include/hssmf.h declares, and rejects malformed input on the host before any
device work (HSSMF_EINVAL)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hssmf.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|void|const char\*)\s+(hssmf_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhssmf.so not built")
    return H.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(H.EXPORTS)


def test_default_options_and_strerror(lib):
    o = H.default_opts()
    assert o.leaf_size == 64 and o.d0 == 128 and o.dd == 128 and o.p == 10 and o.restart == 30
    assert o.tol == 1e-10 and o.rel_tol == 1e-6 and o.min_sep_hss == 2 ** 31 - 1
    assert o.id_kernel == 2 and o.use_graph == 0 and o.hss_update == 1 and o.power_q == 0
    assert o.srrqr_f == 0.0
    assert H.strerror(0) == "ok" and H.strerror(H.HSSMF_ERANK) == "HSS rank exceeds d_max"


def test_measure_peaks_rejects_null_output(lib):
    assert lib.hssmf_measure_peaks(None, None) == H.HSSMF_EINVAL


def test_refactor_device_rejects_null_arguments(lib):
    assert lib.hssmf_refactor_device(None, None) == H.HSSMF_EINVAL


def _call_factor(A_rowptr, A_col, A_val, perm, sep, par, n, opts=None, mem=H.MEM_HOST):
    L = H.load()
    rp = np.ascontiguousarray(A_rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(A_col, dtype=np.int32)
    va = np.ascontiguousarray(A_val, dtype=np.float64)
    pe = np.ascontiguousarray(perm, dtype=np.int32)
    sp = np.ascontiguousarray(sep, dtype=np.int32)
    pa = np.ascontiguousarray(par, dtype=np.int32)
    csr = H.CSRArg(n, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, mem)
    od = H.OrderingArg(pe.ctypes.data, len(pa), sp.ctypes.data, pa.ctypes.data)
    o = opts if opts is not None else H.default_opts()
    h = ctypes.c_void_p()
    rc = L.hssmf_factor(ctypes.byref(csr), ctypes.byref(od), ctypes.byref(o), None, ctypes.byref(h))
    if h:
        L.hssmf_destroy(h)
    return rc


@pytest.fixture(scope="module")
def small():
    A = P.poisson2d(8)
    o = P.geometric_nd((8, 8), 2)
    return A, o


def test_rejects_bad_permutation(lib, small):
    A, o = small
    perm = o.perm.copy()
    perm[3] = perm[4]
    assert _call_factor(A.rowptr, A.colind, A.val, perm, o.sep_ptr, o.parent, A.n) == H.HSSMF_EINVAL


def test_rejects_bad_tree(lib, small):
    A, o = small
    par = o.parent.copy()
    par[0] = 0                                  # not after its child
    assert _call_factor(A.rowptr, A.colind, A.val, o.perm, o.sep_ptr, par, A.n) == H.HSSMF_EINVAL
    sep = o.sep_ptr.copy()
    sep[-1] -= 1                                # does not span [0, n)
    assert _call_factor(A.rowptr, A.colind, A.val, o.perm, sep, o.parent, A.n) == H.HSSMF_EINVAL


def test_rejects_bad_csr(lib, small):
    A, o = small
    col = A.colind.copy()
    col[5] = A.n + 3
    assert _call_factor(A.rowptr, col, A.val, o.perm, o.sep_ptr, o.parent, A.n) == H.HSSMF_EINVAL
    rp = A.rowptr.copy()
    rp[4], rp[5] = rp[5], rp[4]
    assert _call_factor(rp, A.colind, A.val, o.perm, o.sep_ptr, o.parent, A.n) == H.HSSMF_EINVAL


def test_rejects_separator_violation(lib, small):
    """An ordering whose separators do not separate (identity permutation
    with the ND tree) is refused."""
    A, o = small
    assert _call_factor(A.rowptr, A.colind, A.val, np.arange(A.n), o.sep_ptr, o.parent, A.n) == H.HSSMF_EINVAL


def test_rejects_bad_options(lib, small):
    A, o = small
    for field, val in (("leaf_size", 0), ("d0", 0), ("dd", 0), ("restart", 0), ("gemm_prec", 7), ("rel_tol", -1.0), ("id_kernel", 5), ("use_graph", 2), ("gemm_tile", 96),
                       ("abs_tol", -1e-3), ("hss_update", 2), ("keep_stages", 3)):
        opts = H.default_opts(**{field: val})
        assert _call_factor(A.rowptr, A.colind, A.val, o.perm, o.sep_ptr, o.parent, A.n, opts) == H.HSSMF_EINVAL
    # power iteration: at most 4 steps, and only with FP64 products
    for kw in (dict(power_q=-1), dict(power_q=5), dict(power_q=1, gemm_prec="fp32"),
               dict(power_q=2, gemm_prec="bf16")):
        opts = H.default_opts(**kw)
        assert _call_factor(A.rowptr, A.colind, A.val, o.perm, o.sep_ptr, o.parent, A.n, opts) == H.HSSMF_EINVAL, kw
    # strong RRQR: 0 (off) or f > 1 (finite), and only on the resident ID kernel
    for kw in (dict(srrqr_f=-1.0), dict(srrqr_f=0.5), dict(srrqr_f=1.0), dict(srrqr_f=float("nan")),
               dict(srrqr_f=float("inf")), dict(srrqr_f=2.0, id_kernel="stepwise"),
               dict(srrqr_f=2.0, id_kernel="cooperative")):
        opts = H.default_opts(**kw)
        assert _call_factor(A.rowptr, A.colind, A.val, o.perm, o.sep_ptr, o.parent, A.n, opts) == H.HSSMF_EINVAL, kw


def test_batch_rejects_bad_input(lib, small):
    """hssmf_factor_batch: nsys < 1 and a malformed system are refused on the
    host."""
    A, o = small
    keep = []
    good = H._args(A, o, keep)
    bad_perm = o.perm.copy()
    bad_perm[0] = bad_perm[1]

    class _O:
        perm, sep_ptr, parent = bad_perm, o.sep_ptr, o.parent
    bad = H._args(A, _O, keep)
    L = H.load()
    opts = H.default_opts()
    for systems, nsys in (([good], 0), ([good, bad], 2)):
        csrs = (H.CSRArg * len(systems))(*[s[0] for s in systems])
        ords = (H.OrderingArg * len(systems))(*[s[1] for s in systems])
        h = ctypes.c_void_p()
        rc = L.hssmf_factor_batch(nsys, csrs, ords, ctypes.byref(opts), None, ctypes.byref(h))
        if h:
            L.hssmf_destroy(h)
        assert rc == H.HSSMF_EINVAL


def test_rejects_unknown_memory_kind(lib, small):
    """hssmf_csr.mem is HSSMF_MEM_HOST or HSSMF_MEM_DEVICE; anything else is
    refused before the arrays are read."""
    A, o = small
    assert _call_factor(A.rowptr, A.colind, A.val, o.perm, o.sep_ptr, o.parent, A.n, mem=5) == H.HSSMF_EINVAL


def test_solve_family_rejects_bad_arguments(lib):
    """Null handles, negative right-hand-side counts and null vectors are
    refused on the host."""
    buf = np.zeros(4)
    p = ctypes.c_void_p(buf.ctypes.data)
    for fn in (lib.hssmf_solve, lib.hssmf_solve_transpose):
        assert fn(None, 1, p, p, None) == H.HSSMF_EINVAL
    assert lib.hssmf_solve_batch(None, None, None, None) == H.HSSMF_EINVAL


def test_complex_factor_rejects_bad_input(lib):
    """hssmf_factor_z refuses malformed complex input on the host, before any
    device work, and hssmf_refactor_z a null handle."""
    A = P.helmholtz(6, 2, npml=1)
    o = P.geometric_nd((6, 6), 2)
    keep = []

    def call(rowptr, colind, zval, perm, n=A.n, opts=None):
        arrs = (np.ascontiguousarray(rowptr, dtype=np.int64), np.ascontiguousarray(colind, dtype=np.int32),
                np.ascontiguousarray(zval, dtype=np.complex128).view(np.float64),
                np.ascontiguousarray(perm, dtype=np.int32), np.ascontiguousarray(o.sep_ptr, dtype=np.int32),
                np.ascontiguousarray(o.parent, dtype=np.int32))
        keep.append(arrs)
        rp, ci, va, pe, sp, pa = arrs
        csr = H.CSRArg(n, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, H.MEM_HOST)
        ordg = H.OrderingArg(pe.ctypes.data, len(pa), sp.ctypes.data, pa.ctypes.data)
        h = ctypes.c_void_p()
        return lib.hssmf_factor_z(ctypes.byref(csr), ctypes.byref(ordg), ctypes.byref(opts or H.default_opts()),
                                  None, ctypes.byref(h))

    bad_col = A.colind.copy()
    bad_col[3] = A.n
    assert call(A.rowptr, bad_col, A.val, o.perm) == H.HSSMF_EINVAL
    bad_perm = o.perm.copy()
    bad_perm[0] = -1
    assert call(A.rowptr, A.colind, A.val, bad_perm) == H.HSSMF_EINVAL
    assert call(A.rowptr, A.colind, A.val, o.perm, n=-1) == H.HSSMF_EINVAL
    assert call(A.rowptr, A.colind, A.val, o.perm, opts=H.default_opts(srrqr_f=0.5)) == H.HSSMF_EINVAL
    assert lib.hssmf_factor_z(None, None, None, None, None) == H.HSSMF_EINVAL
    assert lib.hssmf_refactor_z(None, None) == H.HSSMF_EINVAL
    assert lib.hssmf_refactor_z_device(None, None) == H.HSSMF_EINVAL
