"""Complex systems on the GPU (the Helmholtz problems of Sec. 6.1, complex
arithmetic): hssmf_factor_z factors the real-equivalent form, against the
oracle's multifrontal method on its own real-equivalent form (ranks per
front equal, M^-1 s and M^-H s to the HSS parity tolerance) and against a
complex sparse direct solve (the solution of A z = s and of A^H z = s);
hssmf_refactor_z with new complex values equals a fresh factorization bit
for bit."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import complexeq as CE
from oracle import mf
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = {
    "h2d48-dense": (lambda: (P.helmholtz(48, 2, npml=8), P.geometric_nd((48, 48), 4)), dict()),
    "h2d48": (lambda: (P.helmholtz(48, 2, npml=8), P.geometric_nd((48, 48), 4)),
              dict(min_sep_hss=64, leaf_size=16, rel_tol=1e-6, d0=32, dd=16, p=8)),
    "h3d14": (lambda: (P.helmholtz(14, 3, npml=4), P.geometric_nd((14, 14, 14), 3)),
              dict(min_sep_hss=128, leaf_size=32, rel_tol=1e-6, d0=64, dd=32, p=8)),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    H.load()


@pytest.mark.parametrize("case,upd", [("h2d48-dense", "dense"), ("h2d48", "dense"), ("h2d48", "lowrank"),
                                      ("h3d14", "dense")])
def test_complex_system_matches_the_oracle(case, upd):
    mk, kw = CASES[case]
    A, o = mk()
    print(f"case {case} {upd}", flush=True)
    ofac = mf.factor(CE.real_form(A), CE.real_ordering(o), mf.Options(**kw))
    fac = H.ZFactorization(A, o, hss_update=upd, tol=1e-12, **kw)
    ranks = [tuple(int(v) for v in r) for r in mf.hss_ranks(ofac)]
    assert fac.hss_ranks() == ranks
    if kw:
        assert ranks, "no HSS front"
    rg = np.random.default_rng(4)
    s = rg.standard_normal(A.n) + 1j * rg.standard_normal(A.n)
    st = torch.tensor(s, device=DEV)
    tol = 1e-12 if not kw else 1e-9
    for tr in (False, True):
        y = fac.apply(st, trans=tr).cpu().numpy()
        yo = CE.to_complex(mf.apply_inverse(ofac, CE.to_real(s), trans=tr))
        assert np.linalg.norm(y - yo) <= tol * np.linalg.norm(yo), (case, upd, tr)
    S = A.to_scipy().tocsc()
    z = spla.spsolve(S, s)
    x, info = fac.solve(st)
    assert info.rel_residual <= 1e-12
    assert np.linalg.norm(x.cpu().numpy() - z) <= 1e-8 * np.linalg.norm(z)
    zh = spla.spsolve(S.conj().T.tocsc(), s)
    xh, info = fac.solve_transpose(st)
    assert np.linalg.norm(xh.cpu().numpy() - zh) <= 1e-8 * np.linalg.norm(zh)
    fac.close()


def test_complex_refactor_equals_a_fresh_factorization():
    """New complex values on the same pattern (another frequency at the same
    spacing): hssmf_refactor_z, and hssmf_refactor_z_device from values in
    device memory, give the factorization hssmf_factor_z gives for them, bit
    for bit."""
    mk, kw = CASES["h2d48"]
    A, o = mk()
    B = P.helmholtz(48, 2, freq=12.0, ppw=12.5, npml=8)
    assert np.array_equal(A.colind, B.colind) and np.array_equal(A.rowptr, B.rowptr)
    s = torch.tensor(np.random.default_rng(6).standard_normal(A.n) + 0j, device=DEV)
    f1 = H.ZFactorization(A, o, **kw)
    f1.refactor(B.val)
    y1 = f1.apply(s).cpu().numpy()
    f1.refactor(torch.tensor(A.val, device=DEV))   # back to A's values, from the device
    f1.refactor(torch.tensor(B.val, device=DEV))
    y1d = f1.apply(s).cpu().numpy()
    f1.close()
    f2 = H.ZFactorization(B, o, **kw)
    y2 = f2.apply(s).cpu().numpy()
    f2.close()
    assert np.array_equal(y1, y2)
    assert np.array_equal(y1d, y2)


def test_complex_system_with_power_iteration_and_strong_rrqr():
    """Every option applies to the real-equivalent form: power iteration
    (q = 1) and the strong RRQR (f = 1.2) together on H2D 48^2, against the
    oracle with the same options (ranks and interchange counts equal,
    M^-1 s to the HSS parity tolerance)."""
    mk, kw = CASES["h2d48"]
    A, o = mk()
    kw = dict(kw, power_q=1, srrqr_f=1.2)
    ofac = mf.factor(CE.real_form(A), CE.real_ordering(o), mf.Options(**kw))
    fac = H.ZFactorization(A, o, **kw)
    assert fac.hss_ranks() == [tuple(int(v) for v in r) for r in mf.hss_ranks(ofac)]
    assert fac.stats()["srrqr_swaps"] == sum(fa.data["H"].stats["swaps"] for fa in ofac.factors if fa.kind == "hss")
    s = np.random.default_rng(8).standard_normal(A.n) + 1j * np.random.default_rng(9).standard_normal(A.n)
    y = fac.apply(torch.tensor(s, device=DEV)).cpu().numpy()
    yo = CE.to_complex(mf.apply_inverse(ofac, CE.to_real(s)))
    assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo)
    fac.close()
