"""Pins for the oracle's HSS toolkit: ID, Alg. 1, matvec / extraction,
ULV factorization and solves, low-rank Schur product (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import hss as H
from oracle.symbolic import hss_tree, HNode


class DenseOp:
    def __init__(self, A):
        self.A = A

    def sample(self, R):
        return self.A @ R, self.A.T @ R

    def extract(self, I, J):
        return self.A[np.ix_(np.asarray(I, int), np.asarray(J, int))]


def _rand_fn(n, seed=0):
    rg = np.random.default_rng(seed)
    cache = {}

    def rand(c0, nc):
        for c in range(c0, c0 + nc):
            if c not in cache:
                cache[c] = rg.standard_normal(n)
        return np.stack([cache[c] for c in range(c0, c0 + nc)], axis=1)
    return rand


def _four_leaf_hss(rng, m=(5, 6, 4, 7), r=3):
    """The 7-node example of Fig. 1 / Eq. HSSexamplematrix with random
    interpolative generators of rank r."""
    lo = np.cumsum((0,) + m)
    nodes = [HNode(lo[0], lo[1]), HNode(lo[1], lo[2]), HNode(lo[0], lo[2], [0, 1]),
             HNode(lo[2], lo[3]), HNode(lo[3], lo[4]), HNode(lo[2], lo[4], [3, 4]),
             HNode(lo[0], lo[4], [2, 5])]
    for p, cs in ((2, (0, 1)), (5, (3, 4)), (6, (2, 5))):
        for c in cs:
            nodes[c].parent = p
    gen = [H.NodeGen() for _ in nodes]
    for t, nd in enumerate(nodes):
        if t == 6:
            continue
        mm = nd.m if nd.leaf else 2 * r
        for side in "UV":
            perm = rng.permutation(mm)
            E = rng.standard_normal((mm - r, r))
            setattr(gen[t], side + "perm", perm)
            setattr(gen[t], side + "E", E)
        if nd.leaf:
            gen[t].D = rng.standard_normal((nd.m, nd.m)) + 4 * np.eye(nd.m)
    for t in (2, 5, 6):
        gen[t].B12 = rng.standard_normal((r, r))
        gen[t].B21 = rng.standard_normal((r, r))
    return H.HSS(nodes, gen, 6)


def _expand_by_formula(hs):
    """Eq. HSSexamplematrix written out block by block."""
    g = hs.gen
    U = [x.U() if x.UE is not None else None for x in g]
    V = [x.V() if x.VE is not None else None for x in g]
    bd = sla.block_diag
    U3 = bd(U[0], U[1]) @ U[2]
    U6 = bd(U[3], U[4]) @ U[5]
    V3 = bd(V[0], V[1]) @ V[2]
    V6 = bd(V[3], V[4]) @ V[5]
    top = np.block([[g[0].D, U[0] @ g[2].B12 @ V[1].T], [U[1] @ g[2].B21 @ V[0].T, g[1].D]])
    bot = np.block([[g[3].D, U[3] @ g[5].B12 @ V[4].T], [U[4] @ g[5].B21 @ V[3].T, g[4].D]])
    return np.block([[top, U3 @ g[6].B12 @ V6.T], [U6 @ g[6].B21 @ V3.T, bot]])


def test_four_leaf_example_expand_matvec_extract(rng):
    hs = _four_leaf_hss(rng)
    F = _expand_by_formula(hs)
    assert np.allclose(H.hss_dense(hs, 6), F, rtol=0, atol=1e-12)
    X = rng.standard_normal((F.shape[0], 3))
    assert np.allclose(H.hss_matvec(hs, 6, X), F @ X, atol=1e-11)
    assert np.allclose(H.hss_matvec(hs, 6, X, trans=True), F.T @ X, atol=1e-11)
    I = np.array([0, 3, 21, 9, 10])
    J = np.array([20, 1, 5, 5])
    assert np.allclose(H.hss_extract(hs, 6, I, J), F[np.ix_(I, J)], atol=1e-12)
    # a subtree (node 5) is the HSS matrix of its block
    lo, hi = hs.nodes[5].lo, hs.nodes[5].hi
    assert np.allclose(H.hss_matvec(hs, 5, X[lo:hi]), F[lo:hi, lo:hi] @ X[lo:hi], atol=1e-11)


def test_id_identities(rng):
    """Y = Y(:,J) X with X(:,J) = I exactly (Sec. 2.2)."""
    Y = rng.standard_normal((30, 8)) @ rng.standard_normal((8, 50))
    perm, E, k = H.interp_decomp(Y, 1e-12)
    assert k == 8
    J = perm[:k]
    X = H.interp_matrix(perm, E).T          # k x m
    assert np.array_equal(X[:, J], np.eye(k))
    assert np.linalg.norm(Y - Y[:, J] @ X) <= 1e-12 * np.linalg.norm(Y)


def test_cpqr_matches_library_on_well_separated_columns(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    Y = Q[:, :12] * np.geomspace(1, 1e-3, 12) @ rng.standard_normal((12, 12))
    Y = Y * np.geomspace(10, 1, 12)
    perm, R, k = H.cpqr_eps(Y, 0.0)
    _, R2, p2 = sla.qr(Y, pivoting=True)
    assert np.array_equal(perm[:6], p2[:6])
    assert np.allclose(np.abs(np.diag(R[:6, :6])), np.abs(np.diag(R2[:6, :6])), rtol=1e-10)


@pytest.mark.parametrize("eps", [1e-3, 1e-7, 1e-11])
def test_epsilon_rank_rule(rng, eps):
    """Rank stops at the first i with |R_{i+1,i+1}| / |R_11| <= eps (Sec. 5.3).
    The prescribed singular values lie two decades apart and eps sits half
    way between two of them, so the rank is known exactly: the column
    pivoted diagonal follows the singular values within a factor of ~7 here
    (over 200 seeds), well inside the decade of margin on either side.  Both
    sides of the rule are checked: the k-th diagonal entry is above
    eps |R_11| and the (k+1)-th (the one that stopped the loop) is not."""
    n = 60
    sv = 10.0 ** -np.arange(0, 24, 2.0)
    U, _ = np.linalg.qr(rng.standard_normal((n, 12)))
    V, _ = np.linalg.qr(rng.standard_normal((n, 12)))
    Y = (U * sv) @ V.T
    _, R, k = H.cpqr_eps(Y, eps)
    expect = int(np.sum(sv > eps))
    assert k == expect
    _, Rf, _ = H.cpqr_eps(Y, 0.0)
    dg = np.abs(np.diag(Rf)) / abs(Rf[0, 0])
    assert dg[k - 1] > eps
    assert dg[k] <= eps


@pytest.mark.parametrize("atol", [3e-3, 3e-7, 3e-11])
def test_absolute_rank_rule(rng, atol):
    """The absolute tolerance: the rank stops at the first i with
    |R_{i+1,i+1}| <= max(eps |R_11|, atol).  The columns here are orthogonal
    with norms 10^0, 10^-2, ..., so column-pivoted QR takes them in order of
    norm and |R_ii| equals the i-th norm (the projections change nothing): the
    rank is exactly the number of norms above atol, with eps far below.  A
    matrix whose largest column is at or below atol has rank 0."""
    n = 40
    nrm = 10.0 ** -np.arange(0, 24, 2.0)
    Q, _ = np.linalg.qr(rng.standard_normal((n, len(nrm))))
    Y = Q * nrm
    Y = Y[:, rng.permutation(len(nrm))]
    _, R, k = H.cpqr_eps(Y, 1e-20, atol)
    assert k == int(np.sum(nrm > atol))
    assert np.allclose(np.abs(np.diag(R))[:k], nrm[:k], rtol=1e-12, atol=0)
    _, _, k0 = H.cpqr_eps(Y * (atol / 2.0), 1e-20, atol)
    assert k0 == 0
    # the relative rule still binds when it is the larger of the two
    _, _, k2 = H.cpqr_eps(Y, 3e-5, 3e-11)
    assert k2 == 3


def test_omega_annihilates_interpolative_basis(rng):
    """Omega U = [0; I] exactly for U = Pi [I; E] (Sec. 2.3)."""
    m, r = 11, 4
    perm = rng.permutation(m)
    E = rng.standard_normal((m - r, r))
    U = H.interp_matrix(perm, E)
    Om = np.block([[-E, np.eye(m - r)], [np.eye(r), np.zeros((r, m - r))]])[:, np.argsort(perm)]
    OU = Om @ U
    assert np.array_equal(OU[:m - r], np.zeros((m - r, r)))
    assert np.array_equal(OU[m - r:], np.eye(r))


def _hss_matrix(rng, n, rank, decay=1.0):
    """A dense matrix with HSS structure: smooth kernel plus diagonal."""
    x = np.sort(rng.uniform(0, 1, n))
    K = 1.0 / (1.0 + 50 * np.abs(x[:, None] - x[None, :])) + 0.3 * np.outer(np.sin(7 * x), np.cos(3 * x))
    return K + n * np.eye(n) * 0.05


def test_compression_exact_recovery(rng):
    """eps -> 0 and d >= m + p: the HSS reproduces the matrix (Alg. 1)."""
    n = 96
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    nodes, k, q = hss_tree(n, 0, 12)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-15, 130, 16, 10, 10000)
    assert np.linalg.norm(H.hss_dense(hs, hs.root) - A) <= 1e-12 * np.linalg.norm(A)


def test_nested_bases_reproduce_offdiagonal_block_rows(rng):
    """Interpolative property of the nested bases (Sec. 2.2, Eq. nestedUV):
    at every non-root node, the off-diagonal block row is its skeleton rows
    mapped through the expanded row basis, A(I, I^c) = U^big A(J^r, I^c),
    and likewise for columns, A(I^c, I) = A(I^c, J^c) (V^big)^T.  The
    transposed product big_t agrees with the expanded basis.  Rows and
    columns are scaled differently so that the row and column bases differ
    (with U in place of V the check misses by ~0.7)."""
    n = 96
    A = _hss_matrix(rng, n, 0)
    A = np.exp(rng.standard_normal(n))[:, None] * A * np.exp(rng.standard_normal(n))[None, :]
    nodes, k, q = hss_tree(n, 0, 12)
    root = len(nodes) - 1
    hs = H.compress(DenseOp(A), nodes, root, _rand_fn(n), 1e-10, 48, 16, 8, 10000)
    X = rng.standard_normal((n, 3))
    checked = 0
    for t, nd in enumerate(hs.nodes):
        if t == root:
            continue
        g = hs.gen[t]
        rows = np.arange(nd.lo, nd.hi)
        comp = np.setdiff1d(np.arange(n), rows)
        Ub = H.down_expand(hs, t, np.eye(g.r), "U")
        Vb = H.down_expand(hs, t, np.eye(g.c), "V")
        blk_r, blk_c = A[np.ix_(rows, comp)], A[np.ix_(comp, rows)]
        assert np.linalg.norm(blk_r - Ub @ A[np.ix_(g.Ir, comp)]) <= 1e-6 * np.linalg.norm(blk_r)
        assert np.linalg.norm(blk_c - A[np.ix_(comp, g.Ic)] @ Vb.T) <= 1e-6 * np.linalg.norm(blk_c)
        for which, G in (("U", Ub), ("V", Vb)):
            assert np.allclose(H.big_t(hs, t, X[rows], which), G.T @ X[rows], rtol=0, atol=1e-12 * np.abs(X).max() * max(1.0, np.abs(G).max()) * len(rows))
        checked += 1
    assert checked == root


def test_compression_b_blocks_are_submatrices(rng):
    """B_{nu1,nu2} = A(I^r_nu1, I^c_nu2) bit-exactly (Sec. 2.2)."""
    n = 80
    A = _hss_matrix(rng, n, 0)
    nodes, k, q = hss_tree(50, 30, 10)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-8, 40, 20, 8, 10000)
    for t, nd in enumerate(nodes):
        if nd.children:
            a, b = nd.children
            assert np.array_equal(hs.gen[t].B12, A[np.ix_(hs.gen[a].Ir, hs.gen[b].Ic)])
            assert np.array_equal(hs.gen[t].B21, A[np.ix_(hs.gen[b].Ir, hs.gen[a].Ic)])
        if nd.leaf:
            assert np.array_equal(hs.gen[t].D, A[nd.lo:nd.hi, nd.lo:nd.hi])


def test_compression_known_ranks(rng):
    """A synthetic HSS matrix with interpolative generators of rank r is
    recovered with rank exactly r at every node when d >= r + p."""
    r = 3
    src = _four_leaf_hss(rng, m=(9, 10, 8, 11), r=r)
    A = H.hss_dense(src, 6)
    hs = H.compress(DenseOp(A), src.nodes, 6, _rand_fn(A.shape[0]), 1e-10, 16, 8, 5, 1000)
    for t in range(6):
        assert hs.gen[t].r == r and hs.gen[t].c == r
    assert np.linalg.norm(H.hss_dense(hs, 6) - A) <= 1e-9 * np.linalg.norm(A)


def test_adaptive_rank_growth(rng):
    """Growth-round count in closed form (Sec. 2.2.1).  The off-diagonal
    blocks of A = (rank 40) + 30 I have rank 40 at the two 60-row nodes and
    the 30-row leaves are full rank.  With d0 = dd = 8, p = 4, a leaf passes
    through k = m once d >= 30 + p.  A 60-row node needs its ID rank 40 <= d - p,
    so d = 8 + 8j >= 44 first holds at d = 48: five growth rounds.  The
    compression is then accurate, and d_max = 47 (one below) is refused."""
    n = 120
    A = (rng.standard_normal((n, 40)) @ rng.standard_normal((40, n))) + 30 * np.eye(n)
    nodes, k, q = hss_tree(60, 60, 30)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-12, 8, 8, 4, 10000)
    assert hs.stats["d"] == 48 and hs.stats["rounds"] == 5
    assert np.linalg.norm(H.hss_dense(hs, hs.root) - A) <= 1e-9 * np.linalg.norm(A)
    assert H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-12, 8, 8, 4, 48).stats["d"] == 48
    for d_max in (47, 24):
        with pytest.raises(H.RankError):
            H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-12, 8, 8, 4, d_max)


@pytest.mark.parametrize("transpose", [False, True])
def test_growth_rule_binds_on_each_side(transpose):
    """The success test k <= d - p (Sec. 2.2.1) holds separately for row and
    column IDs.  A rank-40 off-diagonal block row of leaf 0 (two rank-20
    blocks with independent row spaces, in the sibling leaf and in the other
    half) is seen only by that leaf's row ID: every column ID, and every
    other row ID, meets rank <= 20.  So the row rule alone demands d - 4 >=
    40, i.e. d = 48 after five rounds from d0 = dd = 8, where a rule without
    p would stop at 40.  The transposed matrix puts the same demand on the
    column rule."""
    rg = np.random.default_rng(7)
    n = 240
    A = 30 * np.eye(n)
    A[0:60, 60:120] += rg.standard_normal((60, 20)) @ rg.standard_normal((20, 60))
    A[0:60, 120:180] += rg.standard_normal((60, 20)) @ rg.standard_normal((20, 60))
    if transpose:
        A = A.T.copy()
    nodes, k, q = hss_tree(n, 0, 60)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-12, 8, 8, 4, 10000)
    side = [(hs.gen[t].c, hs.gen[t].r) if transpose else (hs.gen[t].r, hs.gen[t].c) for t in range(len(nodes) - 1)]
    assert side[0] == (40, 0) and max(max(r, c) for r, c in side[1:]) == 20 and max(c for _, c in side) == 20
    assert hs.stats["d"] == 48 and hs.stats["rounds"] == 5
    assert np.linalg.norm(H.hss_dense(hs, hs.root) - A) <= 1e-12 * np.linalg.norm(A)


def test_full_rank_node_succeeds_with_all_its_rows():
    """The other half of the success test (Sec. 2.2.1): a node whose rank
    equals its number of rows succeeds once every row is a skeleton row,
    k = m, without the p extra samples.  Sibling leaves of 30 rows are
    coupled by full-rank blocks, and the two halves by rank-8 blocks.  So the
    leaves bind at k = m = 30 <= d, giving d = 32 after three rounds from
    d0 = dd = 8; without the k = m clause they would need d - 4 >= 30, i.e. 40."""
    rg = np.random.default_rng(11)
    n = 120
    A = 30 * np.eye(n)
    for r0, c0 in ((0, 30), (30, 0), (60, 90), (90, 60)):
        A[r0:r0 + 30, c0:c0 + 30] += rg.standard_normal((30, 30))
    A[0:60, 60:120] += rg.standard_normal((60, 8)) @ rg.standard_normal((8, 60))
    A[60:120, 0:60] += rg.standard_normal((60, 8)) @ rg.standard_normal((8, 60))
    nodes, k, q = hss_tree(n, 0, 30)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-12, 8, 8, 4, 10000)
    ranks = [(hs.gen[t].r, hs.gen[t].c) for t in range(len(nodes) - 1)]
    assert ranks == [(30, 30), (30, 30), (8, 8), (30, 30), (30, 30), (8, 8)]
    assert hs.stats["d"] == 32 and hs.stats["rounds"] == 3
    assert np.linalg.norm(H.hss_dense(hs, hs.root) - A) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("s,u,leaf", [(64, 40, 8), (50, 0, 7), (33, 20, 40)])
def test_ulv_equals_dense_solve(rng, s, u, leaf):
    """ULV solves (and transposed solves) of the compressed F11 equal dense LU
    solves of the expanded HSS matrix; Theta^* Phi equals F21 F11^{-1} F12."""
    n = s + u
    A = _hss_matrix(rng, n, 0) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    nodes, k, q = hss_tree(s, u, leaf)
    hs = H.compress(DenseOp(A), nodes, len(nodes) - 1, _rand_fn(n), 1e-6, 24, 16, 6, 10000)
    Fd = H.hss_dense(hs, hs.root)
    F11 = Fd[:s, :s]
    ulv = H.ulv_factor(hs, k)
    b = rng.standard_normal((s, 2))
    kap = np.linalg.cond(F11)
    assert np.allclose(H.ulv_solve(ulv, b), np.linalg.solve(F11, b), rtol=0, atol=1e-13 * kap * np.abs(np.linalg.solve(F11, b)).max())
    zt = H.ulv_solve_transpose(ulv, b)
    assert np.linalg.norm(F11.T @ zt - b) <= 1e-12 * kap * np.linalg.norm(b)
    if u:
        Th, Ph = H.schur_lowrank(ulv, q)
        S = Fd[s:, :s] @ np.linalg.solve(F11, Fd[:s, s:])
        assert np.linalg.norm(Th @ Ph - S) <= 1e-12 * kap * np.linalg.norm(S)
        ops = H.Front11Ops(hs, k, q)
        z = rng.standard_normal((s, 1))
        x = rng.standard_normal((u, 1))
        assert np.allclose(ops.f21(z), Fd[s:, :s] @ z, atol=1e-11)
        assert np.allclose(ops.f12(x), Fd[:s, s:] @ x, atol=1e-11)
        assert np.allclose(ops.f12t(z), Fd[:s, s:].T @ z, atol=1e-11)
        assert np.allclose(ops.f21t(x), Fd[s:, :s].T @ x, atol=1e-11)


@pytest.mark.parametrize("q", [1, 2])
def test_power_iteration_keeps_exact_recovery(rng, q):
    """Power iteration (samples of (F F^T)^q F and (F^T F)^q F^T, Sec. 2.2)
    spans the same spaces as plain sampling when the off-diagonal blocks
    have exact rank r: every node gets rank exactly r and the HSS form
    reproduces the matrix."""
    r = 3
    src = _four_leaf_hss(rng, m=(9, 10, 8, 11), r=r)
    A = H.hss_dense(src, 6)
    hs = H.compress(DenseOp(A), src.nodes, 6, _rand_fn(A.shape[0]), 1e-10, 16, 8, 5, 1000, power_q=q)
    for t in range(6):
        assert hs.gen[t].r == r and hs.gen[t].c == r
    assert np.linalg.norm(H.hss_dense(hs, 6) - A) <= 1e-9 * np.linalg.norm(A)


def test_compression_with_strong_rrqr_keeps_exact_recovery(rng):
    """Alg. 1 with the strong RRQR (Gu and Eisenstat, rank held fixed)
    inside every ID: on off-diagonal blocks of exact rank r every node keeps
    rank r, the HSS form reproduces the matrix, every interpolation
    coefficient is at most f, and with f close to 1 some ID interchanged
    columns."""
    r, f = 3, 1.01
    src = _four_leaf_hss(rng, m=(9, 10, 8, 11), r=r)
    A = H.hss_dense(src, 6)
    hs = H.compress(DenseOp(A), src.nodes, 6, _rand_fn(A.shape[0]), 1e-10, 16, 8, 5, 1000, srrqr_f=f)
    for t in range(6):
        assert hs.gen[t].r == r and hs.gen[t].c == r
        assert np.max(np.abs(hs.gen[t].UE)) <= f * (1 + 1e-9)
        assert np.max(np.abs(hs.gen[t].VE)) <= f * (1 + 1e-9)
    assert hs.stats["swaps"] > 0
    assert np.linalg.norm(H.hss_dense(hs, 6) - A) <= 1e-9 * np.linalg.norm(A)


@pytest.mark.parametrize("q,rank12,rank21", [(0, 4, 3), (1, 2, 1), (2, 1, 1)])
def test_power_iteration_rank_follows_the_amplified_spectrum(q, rank12, rank21):
    """The ID of the power-iterated samples sees the singular values of an
    off-diagonal block raised to 2q + 1.  With zero diagonal blocks,
    F = [0, A12; A21, 0]: F F^T and F^T F are block diagonal, so leaf 1's
    row samples are (A12 A12^T)^q A12 times Gaussian rows and its column
    samples (A21^T A21)^q A21^T times Gaussian rows, and leaf 2's the other
    way round.  A12 = U diag(10^-2j) V^T and A21 = W diag(10^-3j) Z^T
    (j = 0..7, orthonormal factors) differ, so a product taken with F where
    F^T belongs (or the reverse) mixes the two spectra and changes a rank.
    At eps = 1e-7 the eps-rank (|R_kk| <= eps |R_11|, Sec. 5.3) counts the
    singular values whose (2q + 1)-th power exceeds 1e-7 times the largest,
    every decision a decade or more from eps: 4, 2, 1 for A12 and 3, 1, 1
    for A21 at q = 0, 1, 2."""
    rg = np.random.default_rng(17)
    m = 32
    j = np.arange(8)
    orth = lambda: np.linalg.qr(rg.standard_normal((m, 8)))[0]  # noqa: E731
    A12 = orth() @ np.diag(10.0 ** (-2.0 * j)) @ orth().T
    A21 = orth() @ np.diag(10.0 ** (-3.0 * j)) @ orth().T
    A = np.zeros((2 * m, 2 * m))
    A[:m, m:] = A12
    A[m:, :m] = A21
    nodes, k, qq = hss_tree(2 * m, 0, m)
    root = len(nodes) - 1
    hs = H.compress(DenseOp(A), nodes, root, _rand_fn(2 * m, 5), 1e-7, 24, 8, 4, 1000, power_q=q)
    assert (hs.gen[0].r, hs.gen[0].c) == (rank12, rank21)
    assert (hs.gen[1].r, hs.gen[1].c) == (rank21, rank12)
