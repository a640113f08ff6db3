"""Pins for the oracle's multifrontal solver, outer iterations and adjoint
(CPU only): dense LU on tiny grids, exact solution x = 1 for b = A 1,
eps -> 0 makes MF-HSS exact, transposed solves, adjoint identities."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import dense, krylov, mf
from paper_1502_07405_amd import problems as P


def _dense(A):
    return A.to_scipy().toarray()


@pytest.mark.parametrize("kind", ["p2d", "p3d", "cd2d", "indefinite2d"])
def test_dense_mf_equals_dense_lu(kind, rng):
    """Dense multifrontal factorization (Sec. 3.2) equals a dense solve, and
    so does its transposed solve.  The indefinite case (5-point Laplacian
    shifted by -2.1) makes partial pivoting interchange rows inside the
    fronts, which the diagonally dominant cases never do."""
    if kind == "p2d":
        A, o = P.poisson2d(16), P.geometric_nd((16, 16), 4)
    elif kind == "p3d":
        A, o = P.poisson3d(8), P.geometric_nd((8, 8, 8), 2)
    elif kind == "cd2d":
        A, o = P.convdiff2d(14, 18.0, -6.0), P.geometric_nd((14, 14), 3)
    else:
        A, o = P.poisson2d(16), P.geometric_nd((16, 16), 4)
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        A.val = A.val.copy()
        A.val[rows == A.colind] -= 2.1
    fac = mf.factor(A, o, mf.Options())
    if kind == "indefinite2d":
        moved = [np.any(fa.data["P"] != np.arange(len(fa.data["P"]))) for fa in fac.factors if fa.kind == "dense"]
        assert sum(moved) >= len(moved) // 2
    b = rng.standard_normal((A.n, 2))
    Ad = _dense(A)
    for tr in (False, True):
        x = mf.apply_inverse(fac, b, trans=tr)
        xr = np.linalg.solve(Ad.T if tr else Ad, b)
        assert np.linalg.norm(x - xr) <= 1e-13 * np.linalg.norm(xr)


@pytest.mark.parametrize("s,u", [(12, 7), (9, 0), (5, 11)])
def test_partial_lu_block_identities(rng, s, u):
    """Partial LU of one front (Sec. 3.2) against the block-elimination
    identities: P F11 = L11 U11 with |L11| <= 1 (partial pivoting),
    L11 U12 = P F12, L21 U11 = F21, and the update matrix is the Schur
    complement F22 - F21 F11^{-1} F12, formed here by a plain solve."""
    n = s + u
    F = rng.standard_normal((n, n)) + 0.5 * np.eye(n)
    f = dense.partial_lu(F, s)
    L11 = np.tril(f["lu"], -1) + np.eye(s)
    U11 = np.triu(f["lu"])
    PF = F[f["P"]]
    assert sorted(f["P"]) == list(range(s))
    assert np.abs(L11).max() <= 1.0 + 1e-15
    tol = 1e-12 * np.linalg.norm(F)
    assert np.linalg.norm(L11 @ U11 - PF[:s, :s]) <= tol
    assert np.linalg.norm(L11 @ f["U12"] - PF[:s, s:]) <= tol
    assert np.linalg.norm(f["L21"] @ U11 - F[s:, :s]) <= tol
    schur = F[s:, s:] - F[s:, :s] @ np.linalg.solve(F[:s, :s], F[:s, s:])
    assert np.linalg.norm(f["U"] - schur) <= 1e-10 * max(1.0, np.linalg.norm(schur))


@pytest.mark.filterwarnings("ignore:Diagonal number")
def test_partial_lu_reports_a_singular_front():
    """An exactly singular F11 (a zero column) is reported with its front."""
    F = np.eye(6)
    F[:, 2] = 0.0
    with pytest.raises(dense.SingularFront) as e:
        dense.partial_lu(F, 4, front_id=17)
    assert e.value.front == 17


def test_front_samples_equal_the_assembled_front_times_r():
    """Sampling by skinny extend-add (Eq. FtimesR, Sec. 4.3) equals the
    assembled front times R, and its column samples equal F^T R.  The front is
    assembled through element extraction (Sec. 4.5), a separate code path.
    The children's update matrices are random and nonsymmetric, so a column
    sample taken through U instead of U^T shows."""
    A, o = P.convdiff2d(14, 5.0, 3.0), P.geometric_nd((14, 14), 3)
    Ap = mf.permute_csr(A, np.asarray(o.perm, dtype=np.int64))
    fronts = mf.analyse(Ap, o.sep_ptr, o.parent)
    rg = np.random.default_rng(21)
    updates = {f.id: mf.DenseUpdate(rg.standard_normal((len(f.upd), len(f.upd)))) for f in fronts}
    tested = 0
    for f in fronts:
        if len(f.children) < 2:
            continue
        op = mf.FrontOp(Ap, f, fronts, updates)
        F = op.extract(np.arange(op.n), np.arange(op.n))
        R = rg.standard_normal((op.n, 5))
        Sr, Sc = op.sample(R)
        assert np.allclose(Sr, F @ R, rtol=0, atol=1e-12 * np.abs(F).sum())
        assert np.allclose(Sc, F.T @ R, rtol=0, atol=1e-12 * np.abs(F).sum())
        tested += 1
    assert tested >= 3


def test_restarted_gmres_reaches_the_solution():
    """GMRES(m) with restarts (Sec. 6.1 uses GMRES(30)): with m = 5 the
    solve needs several cycles, and each restart continues from the previous
    cycle's iterate.  The result matches the dense solve at the requested
    residual, and the iteration count exceeds one cycle."""
    rg = np.random.default_rng(3)
    n = 60
    A = np.eye(n) + 0.45 * rg.standard_normal((n, n)) / np.sqrt(n)
    b = rg.standard_normal(n)
    x, its, hist = krylov.gmres(lambda v: A @ v, lambda v: v, b, 1e-10, restart=5, max_it=400)
    xr = np.linalg.solve(A, b)
    assert its > 5 and len(hist) >= 3
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


def test_exact_solution_of_ones_rhs():
    """The paper's right-hand side A [1 ... 1]^T (Sec. 6.1) has solution 1."""
    A, o = P.poisson2d(30), P.geometric_nd((30, 30), 4)
    fac = mf.factor(A, o, mf.Options(min_sep_hss=16, leaf_size=8, rel_tol=1e-3, d0=16, dd=16, p=5))
    b = A.matvec(np.ones(A.n))
    x, its, hist = krylov.gmres(A.matvec, lambda v: mf.apply_inverse(fac, v), b, 1e-12)
    assert np.abs(x - 1).max() < 1e-9


def test_hss_tolerance_to_zero_recovers_direct_solver(rng):
    """eps -> 0: MF-HSS equals MF up to rounding, so refinement converges in
    at most one step."""
    A, o = P.convdiff2d(40, 12.0, 9.0), P.geometric_nd((40, 40), 4)
    fac = mf.factor(A, o, mf.Options(min_sep_hss=12, leaf_size=8, rel_tol=1e-15, d0=16, dd=16, p=5))
    b = rng.standard_normal(A.n)
    xr = np.linalg.solve(_dense(A), b)
    for tr in (False, True):
        x = mf.apply_inverse(fac, b, trans=tr)
        xr = np.linalg.solve(_dense(A).T if tr else _dense(A), b)
        assert np.linalg.norm(x - xr) <= 1e-11 * np.linalg.norm(xr)
    x, its, _ = krylov.refine(A.matvec, lambda v: mf.apply_inverse(fac, v), b, 1e-12)
    assert its <= 1


def test_preconditioned_gmres_and_refinement_converge(rng):
    A, o = P.poisson3d(12), P.geometric_nd((12, 12, 12), 2)
    fac = mf.factor(A, o, mf.Options(min_sep_hss=40, leaf_size=16, rel_tol=1e-2, d0=16, dd=16, p=5))
    b = rng.standard_normal(A.n)
    pc = lambda v: mf.apply_inverse(fac, v)
    xg, itg, hg = krylov.gmres(A.matvec, pc, b, 1e-10)
    assert np.linalg.norm(b - A.matvec(xg)) <= 1e-10 * np.linalg.norm(b)
    xr, itr, hr = krylov.refine(A.matvec, pc, b, 1e-10, max_it=100)
    assert np.linalg.norm(b - A.matvec(xr)) <= 1e-10 * np.linalg.norm(b)
    assert itg <= itr + 1
    with pytest.raises(krylov.NoConvergence):
        krylov.refine(A.matvec, pc, b, 1e-14, max_it=1)


def test_rank_stays_flat_in_2d(rng):
    """2D elliptic fronts have O(1) HSS rank (Table 1): the top front's rank
    barely changes as the grid side doubles."""
    ranks = []
    for n in (48, 96):
        A, o = P.poisson2d(n), P.geometric_nd((n, n), 8)
        fac = mf.factor(A, o, mf.Options(min_sep_hss=32, leaf_size=16, rel_tol=1e-6, d0=32, dd=16, p=10))
        ranks.append(max(r[1] for r in mf.hss_ranks(fac)))
    assert ranks[1] <= ranks[0] + 8


def test_hss_front_starts_from_its_hss_childrens_samples():
    """Eq. (Rmerge), Sec. 4.3: a front's random matrix reuses its HSS
    children's random columns, so it starts with as many as they ended with
    (at least d0) and grows by dd from there; its final d is never below a
    child's, and its growth rounds count from that start."""
    A, o = P.poisson2d(48), P.geometric_nd((48, 48), 4)
    d0, dd = 8, 8
    fac = mf.factor(A, o, mf.Options(min_sep_hss=12, leaf_size=8, rel_tol=1e-6, d0=d0, dd=dd, p=4))
    info = {r[0]: r for r in mf.hss_ranks(fac)}
    kids = {}
    for f, par in enumerate(o.parent):
        if par >= 0:
            kids.setdefault(int(par), []).append(f)
    checked = 0
    for f, (_, _, _, d, rounds) in info.items():
        hk = [info[c][3] for c in kids.get(f, []) if c in info]
        start = max([d0] + hk)
        assert d >= start and d == start + rounds * dd, (f, d, rounds, start)
        checked += bool(hk) and max(hk) > d0
    assert checked > 0   # the case the rule is about occurs here


def test_adjoint_of_a_nonsymmetric_system(rng):
    """The adjoint solves with A^T.  On a convection-diffusion matrix, where
    A^T differs from A, lambda equals the dense A^{-T} g and the gradient
    with respect to b is lambda."""
    A, o = P.convdiff2d(20, 25.0, -15.0), P.geometric_nd((20, 20), 4)
    fac = mf.factor(A, o, mf.Options(min_sep_hss=12, leaf_size=8, rel_tol=1e-8, d0=16, dd=16, p=5))
    b = rng.standard_normal(A.n)
    g = rng.standard_normal(A.n)
    x, lam, dval = oadj.solve_and_adjoint(A, fac, b, lambda x: g, tol=1e-13)
    Ad = _dense(A)
    assert np.linalg.norm(Ad - Ad.T) > 0.1 * np.linalg.norm(Ad)
    lam_ref = np.linalg.solve(Ad.T, g)
    assert np.linalg.norm(lam - lam_ref) <= 1e-10 * np.linalg.norm(lam_ref)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.allclose(dval, -lam_ref[rows] * x[A.colind], rtol=0, atol=1e-9 * np.abs(lam_ref).max() * np.abs(x).max())


def test_refinement_starts_from_the_preconditioned_rhs():
    """Iterative refinement starts from x0 = M^{-1} b: with an exact
    factorization (dense multifrontal) it returns at iteration 0."""
    A, o = P.poisson2d(16), P.geometric_nd((16, 16), 4)
    fac = mf.factor(A, o, mf.Options())
    b = A.matvec(np.ones(A.n))
    x, its, hist = krylov.refine(A.matvec, lambda v: mf.apply_inverse(fac, v), b, 1e-12)
    assert its == 0 and len(hist) == 1
    assert np.abs(x - 1).max() < 1e-12


def test_adjoint_matches_dense(rng):
    """lambda = A^{-T} g, dL/db = lambda, dL/dA_ij = -lambda_i x_j on the
    pattern; checked against dense solves and central differences."""
    n = 10
    kap, _ = P.smoothed_log_kappa(n, seed=4)
    A = P.fv_diffusion3d(n, kap)
    o = P.geometric_nd((n, n, n), 2)
    fac = mf.factor(A, o, mf.Options(min_sep_hss=30, leaf_size=16, rel_tol=1e-8, d0=24, dd=16, p=5))
    b = rng.standard_normal(A.n)
    xs = rng.standard_normal(A.n)
    x, lam, dval = oadj.solve_and_adjoint(A, fac, b, lambda x: 2 * (x - xs), tol=1e-13)
    Ad = _dense(A)
    assert np.linalg.norm(x - np.linalg.solve(Ad, b)) <= 1e-11 * np.linalg.norm(x)
    lam_ref = np.linalg.solve(Ad.T, 2 * (x - xs))
    assert np.linalg.norm(lam - lam_ref) <= 1e-8 * np.linalg.norm(lam_ref)
    # central differences of L = ||x - x*||^2 w.r.t. a few matrix entries
    S = A.to_scipy().tocoo()
    for e in rng.choice(S.nnz, 4, replace=False):
        h = 1e-6 * abs(S.data[e])
        Lv = []
        for sgn in (1, -1):
            M = Ad.copy()
            M[S.row[e], S.col[e]] += sgn * h
            xx = np.linalg.solve(M, b)
            Lv.append(np.sum((xx - xs) ** 2))
        fd = (Lv[0] - Lv[1]) / (2 * h)
        assert abs(fd - dval[e]) <= 1e-5 * max(1.0, abs(fd))


def test_work_counts_dense_fronts_follow_the_table2_model():
    """The algorithmic flop count of an all-dense factorization equals the
    geometric model that reproduces Table 2's multifrontal flops (the same
    fronts, counted from box geometry only)."""
    from oracle import work
    from tests.test_oracle_inputs import _mf_flop_model
    for dims, leaf in (((24, 24), 4), ((10, 9, 8), 2)):
        A = P.poisson2d(*dims) if len(dims) == 2 else P.poisson3d(*dims)
        o = P.geometric_nd(dims, leaf)
        fac = mf.factor(A, o, mf.Options())
        w = work.factorization_work(fac)
        assert abs(w["dense_lu"]["flops"] / _mf_flop_model(dims, leaf) - 1) < 1e-12
        assert w["sampling"]["flops"] == w["id"]["flops"] == 0.0


def test_work_counts_id_closed_forms():
    """The ID count 4dmk - 2k^2(d+m) + 4/3 k^3 + k^2(m-k) reduces to the
    textbook Householder QR counts: 4/3 n^3 for a full-rank n x n block
    (k = m = d), 2 d m^2 - 2/3 m^3 for k = m < d; and every attempt of the
    adaptive loop is counted (a node that failed once contributes twice)."""
    from oracle import hss as H
    from oracle import work
    from oracle.symbolic import hss_tree

    class Op:
        def __init__(self, M):
            self.M = M

        def sample(self, R):
            return self.M @ R, self.M.T @ R

        def extract(self, I, J):
            return self.M[np.ix_(np.asarray(I, int), np.asarray(J, int))]

    rng = np.random.default_rng(3)
    n = 40
    M = rng.standard_normal((n, n)) + n * np.eye(n)
    nodes, k, q = hss_tree(n, 0, 20)
    gen = np.random.default_rng(4)
    Hs = H.compress(Op(M), nodes, len(nodes) - 1, lambda c0, nc: gen.standard_normal((n, nc)), 1e-14, 8, 8, 2, 200)
    # closed forms: 4/3 n^3 for a full-rank square block, 2 d m^2 - 2/3 m^3
    # for a full-column-rank d x m block, and the truncated count is the
    # full one minus the columns it skips
    assert work.id_flops(30, 30, 30) == pytest.approx(4 / 3 * 30 ** 3)
    assert work.id_flops(50, 20, 20) == pytest.approx(2 * 50 * 20 ** 2 - 2 / 3 * 20 ** 3)
    assert work.id_flops(50, 20, 0) == 0.0
    seen = 0
    for (t, d, mr, kr, mc, kc) in Hs.stats["log"]["ids"]:
        for m, kk in ((mr, kr), (mc, kc)):
            if kk == m < d:
                seen += 1
                assert work.id_flops(d, m, kk) == pytest.approx(2 * d * m * m - 2 / 3 * m ** 3)
    assert seen > 0
    # full-rank 20-row leaves start at d = 8: they fail (k = 8 > d - p) and are
    # redone after each growth round until d >= 20 + p
    ids = Hs.stats["log"]["ids"]
    leaf_attempts = [e for e in ids if nodes[e[0]].leaf]
    assert len(leaf_attempts) > 2 and Hs.stats["rounds"] >= 2


def test_refinement_hands_over_to_gmres_when_it_stagnates():
    """Refinement x += M^-1 r diverges when M^-1 = 0.3 I on a 2D Laplacian
    (|1 - 0.3 lambda_max| ~ 1.4 > 1): after two steps whose residual does not
    fall below 0.9 times the previous one it hands over to GMRES(30), which
    still reaches the dense solution.  With an exact preconditioner it
    converges at once and never switches."""
    A = P.poisson2d(8)
    S = A.to_scipy()
    Ad = S.toarray()
    b = np.random.default_rng(11).standard_normal(A.n)
    xr = np.linalg.solve(Ad, b)
    x, its, hist, sw = krylov.refine_or_gmres(lambda v: S @ v, lambda r: 0.3 * r, b, 1e-12, max_it=400)
    assert sw
    k = next(i for i in range(2, len(hist)) if hist[i] > 0.9 * hist[i - 1] and hist[i - 1] > 0.9 * hist[i - 2])
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
    assert np.linalg.norm(b - S @ x) <= 1e-12 * np.linalg.norm(b)
    assert k == 2 and its > k
    x2, its2, _, sw2 = krylov.refine_or_gmres(lambda v: S @ v, lambda r: np.linalg.solve(Ad, r), b, 1e-12)
    assert not sw2 and its2 <= 1
