"""The algebraic front end (host code of the library, no GPU): static
scaling and column permutation (Sec. 3.1, the maximum-product matching of
MC64) and the fill-reducing nested dissection with HSS-ordered separators
(Sec. 3.1, Sec. 4.2).

Pins: the matching's product equals the optimum of the assignment problem
solved by scipy's linear_sum_assignment on -log|a_ij| (a library routine;
exact on small dense problems), the scaled matrix has unit diagonal and no
entry above 1, structurally singular patterns are refused; every ordering
is a separator tree (each coupling of P A P^T lies within a front or between
a front and an ancestor), binary, postordered, with one root; its dense
multifrontal flops stay within those of the geometric nested dissection of
the same grid (the reference ordering of Sec. 6.1); a grid separator
ordered by the length-two-enriched bisection falls into contiguous runs of
the separator line.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linear_sum_assignment

from oracle import symbolic as osym
from paper_1502_07405_amd import hssmf as H
from paper_1502_07405_amd import problems as P


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return P.CSR(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64))


def _tree_ok(A, o):
    assert sorted(o.perm.tolist()) == list(range(A.n))
    nf = len(o.parent)
    assert o.sep_ptr[0] == 0 and o.sep_ptr[-1] == A.n and np.all(np.diff(o.sep_ptr) > 0)
    assert np.sum(o.parent < 0) == 1 and o.parent[-1] == -1
    assert np.all((o.parent == -1) | (o.parent > np.arange(nf)))       # postorder
    assert np.bincount(o.parent[o.parent >= 0], minlength=nf).max() <= 2
    Ap = A.to_scipy()[o.perm][:, o.perm].tocoo()
    front_of = np.repeat(np.arange(nf), np.diff(o.sep_ptr))
    anc = [set() for _ in range(nf)]
    for f in range(nf):
        p = o.parent[f]
        while p >= 0:
            anc[f].add(p)
            p = o.parent[p]
    for i, j in zip(Ap.row, Ap.col):
        fi, fj = front_of[i], front_of[j]
        assert fi == fj or fj in anc[fi] or fi in anc[fj]


def _mf_flops(A, o):
    Ap = osym.permute_csr(A, o.perm)
    return sum(2 / 3 * f.s ** 3 + 2 * f.s ** 2 * f.u + 2 * f.s * f.u ** 2
               for f in osym.analyse(Ap, o.sep_ptr, o.parent))


@pytest.mark.parametrize("trial", range(6))
def test_static_pivoting_is_the_maximum_product_matching(trial):
    rng = np.random.default_rng(trial)
    n = 40
    M = sp.random(n, n, density=0.12, random_state=trial, format="csr")
    M = M + sp.csr_matrix(np.diag(rng.uniform(0.1, 1.0, n)))[rng.permutation(n)]   # one perfect matching at least
    A = _csr(M)
    q, r, c = H.static_pivoting(A)
    D = M.toarray()
    cost = np.where(D != 0, -np.log(np.abs(D) + (D == 0)), 1e6)
    ri, ci = linear_sum_assignment(cost)
    assert np.all(D[ri, ci] != 0)
    assert sorted(q.tolist()) == list(range(n))
    got = np.sum(np.log(np.abs(D[np.arange(n), q])))
    assert abs(got - np.sum(np.log(np.abs(D[ri, ci])))) <= 1e-10 * n
    B = H.apply_static_pivoting(A, q, r, c).to_scipy().toarray()
    assert np.allclose(np.abs(np.diag(B)), 1.0, atol=1e-12, rtol=0)
    assert np.abs(B).max() <= 1.0 + 1e-12
    # the map back: B y = Dr b  <=>  A x = b with x[q] = c[q] y
    b = rng.standard_normal(n)
    y = np.linalg.solve(B, r * b)
    x = np.empty(n)
    x[q] = c[q] * y
    assert np.allclose(D @ x, b, atol=1e-9)


def test_static_pivoting_refuses_structural_singularity():
    # rows 0 and 1 can only take column 0
    M = sp.csr_matrix(np.array([[1.0, 0, 0], [2.0, 0, 0], [1.0, 1.0, 1.0]]))
    with pytest.raises(H.HssmfError) as e:
        H.static_pivoting(_csr(M))
    assert e.value.code == H.HSSMF_ESINGULAR


@pytest.mark.parametrize("kind", ["grid2d", "grid3d", "mesh", "two_parts"])
def test_nested_dissection_is_a_separator_tree(kind):
    if kind == "grid2d":
        A = P.poisson2d(40)
    elif kind == "grid3d":
        A = P.poisson3d(12)
    elif kind == "mesh":
        A, _ = P.knn_mesh(3000, 6, seed=2)
    else:
        G = P.poisson2d(20).to_scipy()
        A = _csr(sp.block_diag([G, G]))
    o = H.nested_dissection(A, 16, 8)
    _tree_ok(A, o)


@pytest.mark.parametrize("dims,leaf", [((48, 48), 4), ((12, 12, 12), 2)])
def test_nested_dissection_fill_is_no_worse_than_geometric(dims, leaf):
    A = P.poisson2d(*dims) if len(dims) == 2 else P.poisson3d(*dims)
    og = P.geometric_nd(dims, leaf)
    oa = H.nested_dissection(A, int(np.prod([leaf] * len(dims))), 16)
    assert _mf_flops(A, oa) <= 1.25 * _mf_flops(A, og)


def test_separator_order_follows_the_separator_line():
    """A 2D grid's top separator is a line of points; ordered by the
    length-two-enriched recursive bisection, every block of sep_leaf
    consecutive indices (an HSS leaf) is a contiguous run of that line."""
    n = 64
    A = P.poisson2d(n)
    o = H.nested_dissection(A, 16, 8)
    top = o.perm[o.sep_ptr[-2]:o.sep_ptr[-1]]
    xy = np.stack([top % n, top // n], 1)
    axis = 0 if np.ptp(xy[:, 0]) > np.ptp(xy[:, 1]) else 1
    pos = xy[:, axis]
    for k in range(0, len(top), 8):
        blk = np.sort(pos[k:k + 8])
        assert blk[-1] - blk[0] == len(blk) - 1, blk
