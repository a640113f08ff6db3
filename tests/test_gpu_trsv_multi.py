"""Triangular solves of long systems on several workgroups per system.

The forward and backward sweeps solve with the F11 factors of the dense
fronts and the top blocks of the HSS fronts.  Systems of at least 256
entries take the multi-workgroup kernel (one cooperative launch) when they
are launched one by one; the same sweeps captured into a HIP graph take the
one-workgroup kernel.  Each entry goes through the same operations in the
same order in both, so the preconditioner applications must agree bitwise,
forward and transposed, with and without row interchanges; the solve must
still reach the residual, and the indefinite case is also checked against
the oracle's dense multifrontal solve."""
import numpy as np
import pytest

from oracle import mf
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _shifted(A, shift):
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    A.val = A.val.copy()
    A.val[rows == A.colind] -= shift
    return A


CASES = {
    # dense fronts up to 784 entries (7-point Laplacian, no interchanges)
    "dense_p3d28": (lambda: (P.poisson3d(28), P.geometric_nd((28, 28, 28), 4)), {}),
    # indefinite: partial pivoting interchanges rows in most fronts
    "indefinite_p3d24": (lambda: (_shifted(P.poisson3d(24), 6.3), P.geometric_nd((24, 24, 24), 4)), {}),
    # HSS fronts above dense fronts of 256 to 511 entries; the HSS fronts'
    # top blocks are solved with the same kernels
    "hss_p3d40": (lambda: (P.poisson3d(40), P.geometric_nd((40, 40, 40), 4)),
                  dict(min_sep_hss=512, leaf_size=64, rel_tol=1e-6, d0=64, dd=64, p=10)),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.mark.parametrize("case", list(CASES))
def test_multi_workgroup_triangular_solves_match_one_workgroup(case):
    mk, kw = CASES[case]
    A, o = mk()
    print(f"case {case}: n {A.n}", flush=True)
    fg = H.Factorization(A, o, use_graph=1, **kw)   # captured sweeps: one workgroup per system
    fe = H.Factorization(A, o, use_graph=0, **kw)   # launched one by one: several per long system
    assert fe.stats()["trsv_multi_ops"] > 0
    rng = np.random.default_rng(21)
    for rep in range(3):
        v = torch.tensor(rng.standard_normal(A.n), device=DEV)
        for tr in (False, True):
            yg = fg.apply(v, trans=tr)
            ye = fe.apply(v, trans=tr)
            assert torch.equal(yg, ye), (case, rep, tr)
    b = rng.standard_normal(A.n)
    x, info = fe.solve(torch.tensor(b, device=DEV))
    assert info.rel_residual <= 1e-10, (case, info.rel_residual)
    if case == "indefinite_p3d24":
        ofac = mf.factor(A, o, mf.Options())
        for tr in (False, True):
            y = fe.apply(torch.tensor(b, device=DEV), trans=tr).cpu().numpy()
            yo = mf.apply_inverse(ofac, b, trans=tr)
            assert np.linalg.norm(y - yo) <= 1e-11 * np.linalg.norm(yo), (case, tr)
    fg.close()
    fe.close()
