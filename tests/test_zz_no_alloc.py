"""hssmf_solve_noalloc against hssmf_solve through the C ABI: the outer
solver's work vectors in the library's static device scratch instead of
allocated memory give bitwise the same solutions and iteration counts (the
same kernels in the same order, sweeps eager on both sides).  Two calls in a
row, the second on a smaller system, so the second call reuses scratch that
holds the first call's data; plus the size limit, refused before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1502_07405_amd import hssmf as H  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = H.load()
    L.hssmf_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(H.Info)]


def _both(fac, B):
    """hssmf_solve and hssmf_solve_noalloc on the device right-hand sides B
    (n x nrhs); returns both solutions and infos."""
    L = H.load()
    nrhs = B.shape[1]
    Bc = B.t().contiguous()
    out = []
    for fn in (L.hssmf_solve, L.hssmf_solve_noalloc):
        X = torch.full_like(Bc, float("nan"))
        infos = (H.Info * nrhs)()
        rc = fn(fac.h, nrhs, ctypes.c_void_p(Bc.data_ptr()), ctypes.c_void_p(X.data_ptr()), infos)
        assert rc == H.HSSMF_OK, rc
        torch.cuda.synchronize()
        out.append((X.t().cpu(), [(i.iterations, i.rel_residual) for i in infos]))
    return out


@pytest.mark.parametrize("outer", ["ir", "gmres"])
def test_noalloc_solve_matches_solve(outer):
    cases = [
        (P.poisson3d(18), P.geometric_nd((18, 18, 18), 2),
         dict(min_sep_hss=64, leaf_size=20, rel_tol=1e-6, d0=24, dd=16, p=6), 3),
        (P.convdiff2d(30, 10.0, -4.0), P.geometric_nd((30, 30), 4),
         dict(min_sep_hss=16, leaf_size=8, rel_tol=1e-4, d0=16, dd=16, p=5), 2),
    ]
    for k, (A, o, kw, nrhs) in enumerate(cases):
        fac = H.Factorization(A, o, outer=outer, tol=1e-12, **kw)
        B = torch.tensor(np.random.default_rng(30 + k).standard_normal((A.n, nrhs)), device=DEV)
        (x1, i1), (x2, i2) = _both(fac, B)
        assert torch.equal(x1, x2), (outer, k)
        assert i1 == i2
        assert all(r <= 1e-12 for _, r in i2)
        fac.close()


def test_noalloc_refuses_too_large_a_workspace():
    """GMRES(200) on 176,400 unknowns needs 203 x 176,400 doubles of scratch,
    more than the 256 MiB array: HSSMF_ETOOBIG, and the output is untouched."""
    A, o = P.poisson2d(420), P.geometric_nd((420, 420), 8)
    fac = H.Factorization(A, o, outer="gmres", restart=200)
    b = torch.ones(A.n, dtype=torch.float64, device=DEV)
    x = torch.zeros_like(b)
    info = H.Info()
    rc = H.load().hssmf_solve_noalloc(fac.h, 1, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.byref(info))
    assert rc == H.HSSMF_ETOOBIG
    assert int(torch.count_nonzero(x)) == 0
    fac.close()
