"""The batch of 256 independent 2D convection-diffusion systems at its stated
recipe (sides uniform in [48, 160] from seed 2, |w| uniform in [0, 20] with
a random angle, 5-point upwind scaled by h^2, geometric nested dissection to
8 x 8 leaves, HSS on separators >= 64, leaf 16, eps 1e-6, d0 = 32,
Delta d = 16, p = 10), factored in one batched handle, against the oracle
run on eight of the systems whose sides span the range.

- FP64 products: each of the eight systems has the oracle's HSS ranks per
  front and M^{-1} b within 1e-9 (equal ranks leave reduction-order
  rounding only).
- FP32 sampling products with FP64 refinement (the recipe's mixed mode):
  every one of the 256 systems reaches ||b_s - A_s x_s|| / ||b_s|| <= 1e-13
  (per-system stopping rule), and the eight systems' solutions agree with
  the oracle's, refined to the same 1e-13, to 1e-8: ||dx|| / ||x|| <=
  2 kappa(A_s) 1e-13 with kappa below 1.1e4 up to side 160.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import krylov, mf  # noqa: E402
from paper_1502_07405_amd import hssmf as H  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402

DEV = "cuda:0"
KW = dict(min_sep_hss=64, leaf_size=16, rel_tol=1e-6, d0=32, dd=16, p=10)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.fixture(scope="module")
def batch():
    systems = P.convdiff_batch(count=256, seed=2, side_lo=48, side_hi=160, wmax=20.0, leaf_side=8)
    sides = np.array([int(round(np.sqrt(A.n))) for A, _, _ in systems])
    order = np.argsort(sides, kind="stable")
    pick = [int(order[q]) for q in np.linspace(0, len(systems) - 1, 8).round().astype(int)]
    oracle = {}
    for s in pick:
        A, o, _ = systems[s]
        oracle[s] = mf.factor(A, o, mf.Options(**KW))
    return systems, sides, pick, oracle


def test_batch_fp64_matches_the_oracle(batch):
    systems, sides, pick, oracle = batch
    assert sides[pick[0]] == 48 and sides[pick[-1]] == 160
    fac = H.BatchFactorization([(A, o) for A, o, _ in systems], **KW)
    ranks = fac.hss_ranks_by_system()
    b = np.concatenate([bj for _, _, bj in systems])
    y = fac.split(fac.apply(torch.tensor(b, device=DEV)).cpu().numpy())
    for s in pick:
        A, o, bj = systems[s]
        assert ranks.get(s, []) == [tuple(int(v) for v in r) for r in mf.hss_ranks(oracle[s])], s
        yo = mf.apply_inverse(oracle[s], bj)
        assert np.linalg.norm(y[s] - yo) <= 1e-9 * np.linalg.norm(yo), s
    fac.close()


def test_batch_mixed_precision_solves_every_system(batch):
    systems, sides, pick, oracle = batch
    fac = H.BatchFactorization([(A, o) for A, o, _ in systems], gemm_prec="fp32", tol=1e-13, max_it=60, **KW)
    xs, info = fac.solve_batch([torch.tensor(bj, device=DEV) for _, _, bj in systems])
    assert info.rel_residual <= 1e-13
    for s, (A, o, bj) in enumerate(systems):
        xh = xs[s].cpu().numpy()
        assert np.linalg.norm(bj - A.to_scipy() @ xh) <= 1e-13 * np.linalg.norm(bj), s
        if s in oracle:
            S = A.to_scipy()
            xo, _, _ = krylov.refine(lambda v: S @ v, lambda r: mf.apply_inverse(oracle[s], r), bj, 1e-13,
                                     max_it=60)
            assert np.linalg.norm(xh - xo) <= 1e-8 * np.linalg.norm(xo), s
    fac.close()
