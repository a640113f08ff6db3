"""Power-iteration sampling on the GPU against the oracle (Sec. 2.2, the
variant the paper describes as an option): with power_q = q the samples are
S^r = (F F^T)^q F R and S^c = (F^T F)^q F^T R, and Alg. 1 takes
R^r = F^T (F F^T)^(q-1) F R on the row side and R^c = F (F^T F)^(q-1) F^T R
on the column side.  Both sides use the same keyed R and the same rule, so
the ranks must be equal front by front and M^-1 b must agree to the HSS
parity tolerance, in both update forms; at a loose tolerance the iterated
samples give ranks no larger than plain sampling."""
import numpy as np
import pytest

from oracle import mf
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    "p3d16": (lambda: (P.poisson3d(16), P.geometric_nd((16, 16, 16), 2)),
              dict(min_sep_hss=64, leaf_size=20, rel_tol=1e-4, d0=24, dd=16, p=6)),
    "cd2d48": (lambda: (P.convdiff2d(48, 15.0, -7.0), P.geometric_nd((48, 48), 4)),
               dict(min_sep_hss=16, leaf_size=8, rel_tol=1e-4, d0=16, dd=16, p=5)),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


def _ranks(fac):
    return [tuple(int(v) for v in r) for r in mf.hss_ranks(fac)]


@pytest.mark.parametrize("case,q,upd", [("p3d16", 1, "dense"), ("p3d16", 1, "lowrank"), ("p3d16", 2, "dense"),
                                        ("cd2d48", 1, "dense")])
def test_power_iteration_matches_the_oracle(case, q, upd):
    mk, kw = CASES[case]
    A, o = mk()
    print(f"case {case} q {q} {upd}", flush=True)
    ofac = mf.factor(A, o, mf.Options(power_q=q, **kw))
    fac = H.Factorization(A, o, power_q=q, hss_update=upd, **kw)
    assert fac.hss_ranks() == _ranks(ofac)
    b = np.random.default_rng(3).standard_normal(A.n)
    for tr in (False, True):
        y = fac.apply(torch.tensor(b, device=DEV), trans=tr).cpu().numpy()
        yo = mf.apply_inverse(ofac, b, trans=tr)
        assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo), (case, q, upd, tr)
    x, info = fac.solve(torch.tensor(b, device=DEV))
    assert info.rel_residual <= 1e-10
    fac.close()


def test_power_iteration_lowers_ranks_at_a_loose_tolerance():
    mk, kw = CASES["p3d16"]
    A, o = mk()
    kw = dict(kw, rel_tol=1e-2)
    f0 = H.Factorization(A, o, **kw)
    r0 = [max(r[1], r[2]) for r in f0.hss_ranks()]
    f0.close()
    f1 = H.Factorization(A, o, power_q=1, **kw)
    r1 = [max(r[1], r[2]) for r in f1.hss_ranks()]
    assert sum(r1) < sum(r0) and all(a <= b for a, b in zip(r1, r0)), (r0, r1)
    f1.close()
