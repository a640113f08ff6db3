"""Pins for complex systems (the Helmholtz problems of Sec. 6.1) on the
oracle side: the real-equivalent form against complex arithmetic itself, the
oracle's multifrontal solver on that form against a complex sparse direct
solve (a library routine), and the Helmholtz generator's stencil (CPU
only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import complexeq as CE
from oracle import mf
from paper_1502_07405_amd import problems as P


@pytest.fixture(scope="module")
def h2d():
    A = P.helmholtz(20, 2, npml=5)
    o = P.geometric_nd((20, 20), 4)
    return A, o


def test_real_form_multiplies_like_the_complex_matrix(h2d):
    """R(A) to_real(z) = to_real(A z) for a random complex z, and
    R(A)^T to_real(z) = to_real(A^H z): the block signs and the
    interleaving."""
    A, _ = h2d
    rg = np.random.default_rng(1)
    z = rg.standard_normal(A.n) + 1j * rg.standard_normal(A.n)
    S = A.to_scipy()
    R = CE.real_form(A).to_scipy()
    assert np.allclose(R @ CE.to_real(z), CE.to_real(S @ z), rtol=0, atol=1e-12 * abs(S).max() * np.abs(z).max())
    assert np.allclose(R.T @ CE.to_real(z), CE.to_real(S.conj().T @ z), rtol=0,
                       atol=1e-12 * abs(S).max() * np.abs(z).max())
    assert np.array_equal(CE.to_complex(CE.to_real(z)), z)


@pytest.mark.parametrize("hss", [False, True])
def test_multifrontal_on_the_real_form_solves_the_complex_system(h2d, hss):
    """The oracle's multifrontal factorization of the real form, with every
    front dense or with HSS fronts at a tight tolerance, applied to
    to_real(s), is to_real of the complex solution from a complex sparse
    LU (scipy's spsolve); the transposed application solves with A^H."""
    A, o = h2d
    rg = np.random.default_rng(2)
    s = rg.standard_normal(A.n) + 1j * rg.standard_normal(A.n)
    S = A.to_scipy().tocsc()
    z = spla.spsolve(S, s)
    zh = spla.spsolve(S.conj().T.tocsc(), s)
    kw = dict(min_sep_hss=16, leaf_size=8, rel_tol=1e-12, d0=16, dd=16, p=5) if hss else {}
    fac = mf.factor(CE.real_form(A), CE.real_ordering(o), mf.Options(**kw))
    if hss:
        assert any(fa.kind == "hss" for fa in fac.factors)
    x = CE.to_complex(mf.apply_inverse(fac, CE.to_real(s)))
    xh = CE.to_complex(mf.apply_inverse(fac, CE.to_real(s), trans=True))
    tol = 1e-12 if not hss else 1e-7
    assert np.linalg.norm(x - z) <= tol * np.linalg.norm(z)
    assert np.linalg.norm(xh - zh) <= tol * np.linalg.norm(zh)


@pytest.mark.parametrize("ndim,n,width", [(2, 14, 9), (3, 7, 27)])
def test_helmholtz_generator_stencil(ndim, n, width):
    """Pattern (9 / 27 points), complex symmetry, a real matrix without
    layers, and the Laplacian part exact on quadratics: two frequencies at
    the same spacing h (freq * ppw fixed) separate the Laplacian from the
    omega^2 term, L = (w2^2 A(w1) - w1^2 A(w2)) / (w2^2 - w1^2), and at
    points whose whole stencil lies in the grid L q = -Lap q exactly for
    q = x^2 + 3 x y - 2 y^2 (+ z^2 - x z in 3D), with x, y, z in metres."""
    A = P.helmholtz(n, ndim, npml=2)
    S = A.to_scipy()
    assert np.diff(A.rowptr).max() == width
    assert abs(S - S.T).max() == 0.0
    assert np.abs(S.imag).max() > 0
    f1, f2 = 10.0, 14.0
    A1 = P.helmholtz(n, ndim, freq=f1, ppw=15.0, npml=0).to_scipy()
    A2 = P.helmholtz(n, ndim, freq=f2, ppw=15.0 * f1 / f2, npml=0).to_scipy()
    assert abs(A1.imag).max() == 0.0
    w1, w2 = 2 * np.pi * f1, 2 * np.pi * f2
    L = ((w2 ** 2) * A1 - (w1 ** 2) * A2) / (w2 ** 2 - w1 ** 2)
    h = 1500.0 / (f1 * 15.0)
    idx = np.arange(n ** ndim)
    c = [(idx // n ** a) % n * h for a in range(ndim)]
    if ndim == 2:
        q = c[0] ** 2 + 3 * c[0] * c[1] - 2 * c[1] ** 2
        lap = 2.0 - 4.0
    else:
        q = c[0] ** 2 + 3 * c[0] * c[1] - 2 * c[1] ** 2 + c[2] ** 2 - c[0] * c[2]
        lap = 2.0 - 4.0 + 2.0
    inner = np.ones(idx.size, dtype=bool)
    for a in range(ndim):
        g = (idx // n ** a) % n
        inner &= (g > 0) & (g < n - 1)
    Lq = (L @ q.astype(np.complex128)).real
    assert np.allclose(Lq[inner], -lap, rtol=0, atol=1e-9 * np.abs(q).max() / h ** 2)
