"""The algebraic front end ahead of the GPU factorization (Sec. 3.1,
Sec. 4.2): an unstructured-mesh operator (random points, k-nearest-neighbour
graph, nonsymmetric) with its rows scrambled, so that most diagonal entries
are zero, is scaled and column-permuted by static pivoting (MC64's
maximum-product matching), ordered by the library's nested dissection with
HSS-ordered separators, factored on the GPU with HSS fronts, and compared
with the oracle's factorization of the same transformed matrix: equal ranks
per HSS front, M^{-1} v to 1e-9 (rounding only at equal ranks), and the
solution mapped back solves the original system to 1e-10."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import mf  # noqa: E402
from paper_1502_07405_amd import hssmf as H  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.mark.parametrize("upd", ["dense", "lowrank"])
def test_unstructured_mesh_through_the_algebraic_front_end(upd):
    A0, _ = P.knn_mesh(16000, 6, seed=4)
    A = P.permute_rows(A0, seed=5)
    assert np.count_nonzero(A.to_scipy().diagonal()) < A.n // 10
    q, r, c = H.static_pivoting(A)
    B = H.apply_static_pivoting(A, q, r, c)
    o = H.nested_dissection(B, 32, 16)
    kw = dict(min_sep_hss=48, leaf_size=16, rel_tol=1e-6, d0=32, dd=16, p=10)
    ofac = mf.factor(B, o, mf.Options(**kw))
    orr = [tuple(int(v) for v in t) for t in mf.hss_ranks(ofac)]
    assert len(orr) >= 3, "the ordering should give several HSS fronts"
    fac = H.Factorization(B, o, tol=1e-12, max_it=50, hss_update=upd, **kw)
    assert fac.hss_ranks() == orr
    v = np.random.default_rng(7).standard_normal(A.n)
    y = fac.apply(torch.tensor(v, device=DEV)).cpu().numpy()
    yo = mf.apply_inverse(ofac, v)
    assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo)
    b = np.random.default_rng(8).standard_normal(A.n)
    yb, info = fac.solve(torch.tensor(r * b, device=DEV))
    x = np.empty(A.n)
    x[q] = c[q] * yb.cpu().numpy()
    rel = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    print(f"HSS fronts {len(orr)}, ranks {[t[1] for t in orr]}, iterations {info.iterations}, residual {rel:.2e}")
    assert rel <= 1e-10
    fac.close()
