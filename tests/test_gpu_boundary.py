"""The C-ABI's solve family and input forms on the GPU, against the oracle:
several right-hand sides per call, host or device vectors, the per-system
batch solve, a CSR matrix handed over in device memory, and the absolute
compression tolerance.

Solution differences are checked with both sides refined to a relative
residual of 1e-12: then ||x_gpu - x_orc|| / ||x|| <= 2 kappa(A) 1e-12, and
kappa stays below 1e3 for these conv-diff and Poisson cases, so 1e-8 has
a margin of five.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import krylov, mf  # noqa: E402
from paper_1502_07405_amd import hssmf as H  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402

DEV = "cuda:0"
KW = dict(min_sep_hss=16, leaf_size=8, rel_tol=1e-6, d0=16, dd=16, p=5)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.fixture(scope="module")
def cd48():
    A, o = P.convdiff2d(48, 15.0, -7.0), P.geometric_nd((48, 48), 4)
    return A, o, mf.factor(A, o, mf.Options(**KW))


def _oracle_solve(A, ofac, b, trans=False):
    S = A.to_scipy()
    M = S.T if trans else S
    x, _, _ = krylov.refine(lambda z: M @ z, lambda r: mf.apply_inverse(ofac, r, trans=trans), b, 1e-12)
    return x


def test_several_right_hand_sides_match_the_oracle(cd48):
    """nrhs = 3 in one hssmf_solve call (n x 3, device) and nrhs = 2 in one
    hssmf_solve_transpose call: every column within 1e-8 of the oracle's
    solution, and bitwise equal to the same column solved alone."""
    A, o, ofac = cd48
    fac = H.Factorization(A, o, tol=1e-12, **KW)
    B = np.random.default_rng(21).standard_normal((A.n, 3))
    X, infos = fac.solve(torch.tensor(B, device=DEV))
    assert X.shape == (A.n, 3) and len(infos) == 3
    for j in range(3):
        xo = _oracle_solve(A, ofac, B[:, j])
        xj = X[:, j].cpu().numpy()
        assert np.linalg.norm(xj - xo) <= 1e-8 * np.linalg.norm(xo), j
        assert infos[j].rel_residual <= 1e-12
        x1, _ = fac.solve(torch.tensor(B[:, j], device=DEV))
        assert torch.equal(x1.cpu(), X[:, j].cpu()), j
    L, _ = fac.solve_transpose(torch.tensor(B[:, :2], device=DEV))
    for j in range(2):
        lo = _oracle_solve(A, ofac, B[:, j], trans=True)
        assert np.linalg.norm(L[:, j].cpu().numpy() - lo) <= 1e-8 * np.linalg.norm(lo), j
    fac.close()


def test_host_vectors_give_the_device_result(cd48):
    """Host (numpy) right-hand sides and solutions: staged through device
    memory, bitwise the result of the device call."""
    A, o, _ = cd48
    fac = H.Factorization(A, o, **KW)
    B = np.random.default_rng(22).standard_normal((A.n, 2))
    Xh, ih = fac.solve(B)
    assert isinstance(Xh, np.ndarray) and Xh.shape == B.shape
    Xd, idv = fac.solve(torch.tensor(B, device=DEV))
    assert np.array_equal(Xh, Xd.cpu().numpy())
    assert [i.iterations for i in ih] == [i.iterations for i in idv]
    fac.close()


def test_solve_batch_matches_the_oracle():
    """hssmf_solve_batch with one right-hand side per system, host and device
    arrays mixed: every system's x within 1e-8 of the oracle's solution of
    that system alone, and bitwise the packed hssmf_solve result."""
    systems = P.convdiff_batch(count=4, seed=2, side_lo=20, side_hi=40, leaf_side=4)
    kw = dict(KW, tol=1e-12)
    fac = H.BatchFactorization([(A, o) for A, o, _ in systems], **kw)
    bs = [torch.tensor(bj, device=DEV) if s % 2 else bj for s, (_, _, bj) in enumerate(systems)]
    xs, info = fac.solve_batch(bs)
    assert info.rel_residual <= 1e-12
    packed, _ = fac.solve(torch.tensor(np.concatenate([bj for _, _, bj in systems]), device=DEV))
    parts = fac.split(packed.cpu().numpy())
    for s, (A, o, bj) in enumerate(systems):
        xg = xs[s].cpu().numpy() if s % 2 else xs[s]
        assert isinstance(xs[s], torch.Tensor) == bool(s % 2)
        assert np.array_equal(xg, parts[s]), s
        ofac = mf.factor(A, o, mf.Options(**KW))
        xo = _oracle_solve(A, ofac, bj)
        assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo), s
    fac.close()


def test_device_csr_factorization_equals_host_csr(cd48):
    """hssmf_csr.mem = HSSMF_MEM_DEVICE: the same factorization, bitwise, as
    from host arrays."""
    A, o, _ = cd48
    b = torch.tensor(np.random.default_rng(23).standard_normal(A.n), device=DEV)
    out = []
    for dev in (False, True):
        fac = H.Factorization(A, o, device_csr=dev, **KW)
        out.append((fac.hss_ranks(), fac.apply(b).cpu()))
        fac.close()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])


def test_absolute_tolerance_matches_the_oracle():
    """abs_tol large enough to bind (it cuts ranks below the relative rule's)
    gives the oracle's ranks per HSS front, and M^-1 b within 1e-9 of the
    oracle's."""
    A, o = P.poisson3d(16), P.geometric_nd((16, 16, 16), 2)
    kw = dict(min_sep_hss=64, leaf_size=20, rel_tol=1e-8, d0=24, dd=16, p=6)
    loose = mf.factor(A, o, mf.Options(**kw))
    ofac = mf.factor(A, o, mf.Options(abs_tol=1e-4, **kw))
    rk = [tuple(int(v) for v in r) for r in mf.hss_ranks(ofac)]
    assert sum(r[1] for r in rk) < sum(r[1] for r in mf.hss_ranks(loose))
    fac = H.Factorization(A, o, abs_tol=1e-4, **kw)
    assert fac.hss_ranks() == rk
    b = np.random.default_rng(24).standard_normal(A.n)
    y = fac.apply(torch.tensor(b, device=DEV)).cpu().numpy()
    yo = mf.apply_inverse(ofac, b)
    assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo)
    fac.close()
