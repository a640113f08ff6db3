"""Strong rank-revealing QR inside the IDs on the GPU against the oracle
(Gu and Eisenstat with the rank held fixed; Sec. 2.2 and Sec. 7 name it as
the replacement of the column-pivoted QR).  The rank of every ID comes from
the pivoted QR; then, while some interchange of a selected and a remaining
column multiplies |det R11| by more than f, the largest is made and the QR
redone in that pivot order.  Both sides take the same decisions in FP64, so
the ranks and the number of interchanges must be equal and M^-1 b must
agree to the HSS parity tolerance, in both update forms; with f above every
interpolation coefficient nothing changes, bit for bit."""
import numpy as np
import pytest

from oracle import mf
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    # single-workgroup IDs
    "p3d16": (lambda: (P.poisson3d(16), P.geometric_nd((16, 16, 16), 2)),
              dict(min_sep_hss=64, leaf_size=20, rel_tol=1e-4, d0=24, dd=16, p=6)),
    "cd2d48": (lambda: (P.convdiff2d(48, 15.0, -7.0), P.geometric_nd((48, 48), 4)),
               dict(min_sep_hss=16, leaf_size=8, rel_tol=1e-4, d0=16, dd=16, p=5)),
    # IDs of up to 328 rows at 192 samples: three workgroups of one
    # cooperative launch per ID, in the forced re-factorizations too
    "p3d24": (lambda: (P.poisson3d(24), P.geometric_nd((24, 24, 24), 4)),
              dict(min_sep_hss=200, leaf_size=48, rel_tol=1e-9, d0=128, dd=64, p=8)),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


def _ranks(fac):
    return [tuple(int(v) for v in r) for r in mf.hss_ranks(fac)]


def _swaps(fac):
    return sum(fa.data["H"].stats["swaps"] for fa in fac.factors if fa.kind == "hss")


@pytest.mark.parametrize("case,f,upd", [("p3d16", 1.2, "dense"), ("p3d16", 1.2, "lowrank"), ("p3d16", 1.05, "dense"),
                                        ("cd2d48", 1.05, "dense"), ("p3d24", 1.2, "dense")])
def test_strong_rrqr_matches_the_oracle(case, f, upd):
    mk, kw = CASES[case]
    A, o = mk()
    print(f"case {case} f {f} {upd}", flush=True)
    ofac = mf.factor(A, o, mf.Options(srrqr_f=f, **kw))
    fac = H.Factorization(A, o, srrqr_f=f, hss_update=upd, **kw)
    sw = _swaps(ofac)
    assert sw > 0
    assert fac.hss_ranks() == _ranks(ofac)
    assert fac.stats()["srrqr_swaps"] == sw
    b = np.random.default_rng(3).standard_normal(A.n)
    for tr in (False, True):
        y = fac.apply(torch.tensor(b, device=DEV), trans=tr).cpu().numpy()
        yo = mf.apply_inverse(ofac, b, trans=tr)
        assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo), (case, f, upd, tr)
    x, info = fac.solve(torch.tensor(b, device=DEV))
    assert info.rel_residual <= 1e-10
    fac.close()


def test_large_f_changes_nothing():
    """f = 2 is above every interpolation coefficient of the pivoted QR on
    this workload (the oracle makes no interchange): the factorization is
    the one without the strong RRQR, bit for bit."""
    mk, kw = CASES["p3d16"]
    A, o = mk()
    assert _swaps(mf.factor(A, o, mf.Options(srrqr_f=2.0, **kw))) == 0
    b = torch.tensor(np.random.default_rng(5).standard_normal(A.n), device=DEV)
    f0 = H.Factorization(A, o, **kw)
    y0 = f0.apply(b).cpu().numpy()
    f0.close()
    f1 = H.Factorization(A, o, srrqr_f=2.0, **kw)
    assert f1.stats()["srrqr_swaps"] == 0
    y1 = f1.apply(b).cpu().numpy()
    f1.close()
    assert np.array_equal(y0, y1)
