"""GPU parity cases beyond the M-matrix workloads.  Dense fronts with real
row interchanges: the dense-front parity
cases are M-matrices, whose fronts never pivot, so here the 5-point and
7-point Laplacians are shifted to be indefinite, which makes partial
pivoting interchange rows in most fronts, including fronts larger than one
128-column block of the blocked LU.  The adjoint on a nonsymmetric
matrix, where A^T differs from A.  GMRES(2), so that the restart update runs
(the GMRES(30) parity case converges within one cycle)."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import krylov, mf
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _shifted(A, shift):
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    A.val = A.val.copy()
    A.val[rows == A.colind] -= shift
    return A


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_dense_fronts_with_row_interchanges_match_the_oracle(case):
    if case == "2d":
        A, o = _shifted(P.poisson2d(40), 2.1), P.geometric_nd((40, 40), 4)
    else:
        A, o = _shifted(P.poisson3d(14), 6.3), P.geometric_nd((14, 14, 14), 2)
    ofac = mf.factor(A, o, mf.Options())
    moved = [np.any(fa.data["P"] != np.arange(len(fa.data["P"]))) for fa in ofac.factors if fa.kind == "dense"]
    assert sum(moved) >= len(moved) // 2
    fac = H.Factorization(A, o)
    b = np.random.default_rng(5).standard_normal(A.n)
    for tr in (False, True):
        y = fac.apply(torch.tensor(b, device="cuda:0"), trans=tr).cpu().numpy()
        yo = mf.apply_inverse(ofac, b, trans=tr)
        assert np.linalg.norm(y - yo) <= 1e-11 * np.linalg.norm(yo), (case, tr)
    fac.close()


def test_adjoint_of_a_nonsymmetric_system_matches_the_oracle():
    A, o = P.convdiff2d(40, 25.0, -15.0), P.geometric_nd((40, 40), 4)
    kw = dict(min_sep_hss=12, leaf_size=8, rel_tol=1e-8, d0=16, dd=16, p=5)
    ofac = mf.factor(A, o, mf.Options(**kw))
    rg = np.random.default_rng(6)
    b = rg.standard_normal(A.n)
    g = rg.standard_normal(A.n)
    xo, lamo, dvalo = oadj.solve_and_adjoint(A, ofac, b, lambda x: g, tol=1e-13)
    fac = H.Factorization(A, o, tol=1e-13, **kw)
    x, _ = fac.solve(torch.tensor(b, device="cuda:0"))
    db, dval, _ = fac.adjoint(x, torch.tensor(g, device="cuda:0"))
    assert np.linalg.norm(db.cpu().numpy() - lamo) <= 1e-8 * np.linalg.norm(lamo)
    assert np.linalg.norm(dval.cpu().numpy() - dvalo) <= 1e-8 * np.linalg.norm(dvalo)
    fac.close()


def test_gmres_with_restarts_matches_the_oracle():
    w = P.WORKLOADS["poisson2d_100"]
    A, o, b = P.workload(**w)
    kw = dict(min_sep_hss=64, leaf_size=16, rel_tol=1e-2, d0=32, dd=16, p=10)
    S = A.to_scipy()
    ofac = mf.factor(A, o, mf.Options(**kw))
    xo, its, hist = krylov.gmres(lambda v: S @ v, lambda v: mf.apply_inverse(ofac, v), b, 1e-12, restart=2, max_it=200)
    assert len(hist) >= 3   # several cycles
    fac = H.Factorization(A, o, outer="gmres", restart=2, tol=1e-12, max_it=200, **kw)
    x, info = fac.solve(torch.tensor(b, device="cuda:0"))
    x = x.cpu().numpy()
    assert np.linalg.norm(b - S @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)
    assert abs(info.iterations - its) <= 2
    fac.close()
