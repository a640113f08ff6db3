"""Stage-by-stage errors of the GPU factorization against the FP64 oracle,
in FP64 and in the mixed mode (FP32 sampling and Schur-expansion products;
ranks, ULV and refinement in FP64), on Poisson 32^3 with the parameters of
the 64^3 workload (HSS on separators >= 512, leaf 64, eps 1e-6,
d0 = dd = 128, p = 10): two HSS fronts, one of them with an update set.

Per HSS front (hssmf_front_data with keep_stages = 1):
- the samples S^r = F R and S^c = F^T R on the columns both sides drew;
- the ranks and final sample counts;
- the low-rank Schur product Theta^* Phi and the update matrix
  F22 - Theta^* Phi handed to the parent;
and M^{-1} v for v = default_rng(7).  Both forms of an HSS child's update
matrix are run: low rank (the parent samples it by an HSS matrix-vector
product of F22 minus Theta^*(Phi X), in FP64 in either mode, and reads its
entries from the generators) and the dense expansion.

Bounds.  FP64: the same ranks as the oracle, samples to 1e-12 (rounding
only), Schur factors, update and M^{-1} v to 1e-9.  Mixed: the samples
carry the rounding of R and of the children's update matrices to FP32 and
FP32 sums over 32-term k-tiles: |dS| <= (2 u32 + 32 u32) |F| |R| entrywise,
u32 = 2^-24, so ||dS||_F <= 2.1e-6 || |F| |R| ||_F, and || |F| |R| ||_F
stays below 4 ||F R||_F for these diagonally dominant fronts: 1e-5.  The
Schur product, update and M^{-1} v then differ from the oracle's by the
two sides' truncations at eps, amplified by the conditioning of the
fronts (kappa < 1e3 here): 1e-3 for all three.  Ranks are printed, not
bounded (pivots near eps |R_11| may move).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import mf  # noqa: E402
from paper_1502_07405_amd import hssmf as H  # noqa: E402
from paper_1502_07405_amd import problems as P  # noqa: E402

DEV = "cuda:0"
KW = dict(min_sep_hss=512, leaf_size=64, rel_tol=1e-6, d0=128, dd=128, p=10)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.fixture(scope="module")
def case():
    A, o = P.poisson3d(32), P.geometric_nd((32, 32, 32), 4)
    rec = {}
    ofac = mf.factor(A, o, mf.Options(**KW), record=rec)
    return A, o, ofac, rec


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


@pytest.mark.parametrize("prec,upd", [("fp64", "lowrank"), ("fp32", "lowrank"), ("fp64", "dense"), ("fp32", "dense")])
def test_stage_errors_against_the_oracle(case, prec, upd):
    A, o, ofac, rec = case
    fac = H.Factorization(A, o, keep_stages=1, gemm_prec=prec, hss_update=upd, **KW)
    gr = {r[0]: r for r in fac.hss_ranks()}
    orr = {r[0]: r for r in mf.hss_ranks(ofac)}
    assert sorted(gr) == sorted(orr) == sorted(rec)
    lim_s = 1e-12 if prec == "fp64" else 1e-5
    lim_x = 1e-9 if prec == "fp64" else 1e-3
    print(f"\n[{prec} {upd}] front  rank gpu/orc   d gpu/orc   dS^r      dS^c      d(Theta*Phi)  dU")
    for f in sorted(rec):
        r = rec[f]
        Sr = fac.front_data(f, "samples_row")
        Sc = fac.front_data(f, "samples_col")
        dc = min(Sr.shape[1], r["d"])
        So_r, So_c = r["op"].sample(r["rand"](0, dc))
        es_r = _rel(Sr[:, :dc], So_r)
        es_c = _rel(Sc[:, :dc], So_c)
        line = f"{f:6d}  {gr[f][1]:5d}/{orr[f][1]:<5d} {gr[f][3]:5d}/{orr[f][3]:<5d} {es_r:.2e}  {es_c:.2e}"
        assert es_r <= lim_s and es_c <= lim_s, (f, es_r, es_c)
        if r["Theta"] is not None:
            tp = fac.front_data(f, "theta_t").T @ fac.front_data(f, "phi")
            ep = _rel(tp, r["Theta"] @ r["Phi"])
            eu = _rel(fac.front_data(f, "update"), r["update"].dense())
            line += f"  {ep:.2e}      {eu:.2e}"
            assert ep <= lim_x and eu <= lim_x, (f, ep, eu)
        print(line)
    if prec == "fp64":
        assert [gr[f] for f in sorted(gr)] == [tuple(int(v) for v in orr[f]) for f in sorted(orr)]
    v = np.random.default_rng(7).standard_normal(A.n)
    y = fac.apply(torch.tensor(v, device=DEV)).cpu().numpy()
    ey = _rel(y, mf.apply_inverse(ofac, v))
    print(f"[{prec} {upd}] ||dM^-1 v|| / ||M^-1 v|| = {ey:.2e}")
    assert ey <= lim_x
    fac.close()
