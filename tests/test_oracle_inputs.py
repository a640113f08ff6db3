"""Pins for the oracle's RNG, the input generators, the ordering and the
symbolic analysis (CPU only)."""
import os

import numpy as np
import pytest

from oracle import rng as orng
from oracle import symbolic as osym
from oracle import dense as odense
from paper_1502_07405_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_philox_known_answers():
    for row in _rows("philox4x32_10_kat.txt"):
        v = [int(t, 16) for t in row]
        out = orng.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_gaussian_moments_and_keying():
    g = orng.gaussian(7, np.arange(40000), 8)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1) < 0.01
    assert abs((g ** 4).mean() - 3) < 0.05
    # keyed by (seed, row, column): any subset of rows/columns sees the same values
    sub = orng.gaussian(7, np.array([5, 17, 3]), 3, col0=4)
    assert np.array_equal(sub, g[[5, 17, 3]][:, 4:7])
    assert not np.allclose(orng.gaussian(8, np.arange(4), 4), g[:4, :4])


def _mf_flop_model(dims, leaf):
    """sum 2/3 s^3 + 2 s^2 u + 2 s u^2 over the geometric ND fronts, computed
    from box geometry only (separator = cut plane, update = box halo)."""
    tot = 0.0

    def rec(lo, hi):
        nonlocal tot
        ext = [h - l for l, h in zip(lo, hi)]
        if min(ext) <= 0:
            return
        if max(ext) <= leaf:
            s = int(np.prod(ext))
        else:
            ax = int(np.argmax(ext))
            cut = lo[ax] + (ext[ax] - 1) // 2
            hl = list(hi); hl[ax] = cut
            lr = list(lo); lr[ax] = cut + 1
            rec(lo, hl); rec(lr, hi)
            s = int(np.prod([e for b, e in enumerate(ext) if b != ax]))
        u = P.halo_size((lo, hi), dims)
        tot += 2 / 3 * s ** 3 + 2 * s * s * u + 2 * s * u * u
    rec([0] * len(dims), list(dims))
    return tot


def test_nd_flop_model_matches_table2():
    """Table 2 prints the dense-MF factor flops of the geometric-ND runs; our
    ND rule must reproduce them (4.9e12 at 5000^2, 50.0e12 at 125^3)."""
    for kind, dims, leaf, flops in _rows("table2_mf_flops.txt"):
        dims = tuple(int(x) for x in dims.split(","))
        model = _mf_flop_model(dims, int(leaf))
        assert abs(model / float(flops) - 1) < 0.02, (kind, model)


@pytest.mark.parametrize("dims,leaf", [((12, 9), 3), ((7, 8, 6), 2), ((16, 16), 4)])
def test_nd_is_a_separator_tree(dims, leaf):
    o = P.geometric_nd(dims, leaf)
    N = int(np.prod(dims))
    assert sorted(o.perm.tolist()) == list(range(N))
    A = (P.poisson2d(*dims) if len(dims) == 2 else P.poisson3d(*dims)).to_scipy()
    Ap = A[o.perm][:, o.perm].tocoo()
    front_of = np.repeat(np.arange(o.nfront), np.diff(o.sep_ptr))
    anc = [set() for _ in range(o.nfront)]
    for f in range(o.nfront):
        p = o.parent[f]
        while p >= 0:
            anc[f].add(p)
            p = o.parent[p]
    # every coupling is within a front or between a front and an ancestor
    for i, j in zip(Ap.row, Ap.col):
        fi, fj = front_of[i], front_of[j]
        assert fi == fj or fj in anc[fi] or fi in anc[fj]


@pytest.mark.parametrize("dims,leaf", [((20, 20), 4), ((9, 10, 8), 2)])
def test_update_sets_equal_box_halo(dims, leaf):
    """Symbolic update sets (sparse structure) equal the geometric halo of each
    front's subtree box for a 5/7-point stencil."""
    o = P.geometric_nd(dims, leaf)
    A = P.poisson2d(*dims) if len(dims) == 2 else P.poisson3d(*dims)
    Ap = osym.permute_csr(A, o.perm)
    fronts = osym.analyse(Ap, o.sep_ptr, o.parent)
    for f in fronts:
        assert f.u == P.halo_size(o.boxes[f.id], dims)
        assert np.all(f.upd >= f.sep_hi)


def test_extend_add_worked_example():
    """Eq. extend-add: U1 on {1,2} and U2 on {1,3} sum to the printed 3x3."""
    sym = {}
    vals = iter(np.arange(1.0, 9.0) * 10.0 + np.arange(8) * 0.125)
    for k in (1, 2):
        for nm in "abcd":
            sym[f"{nm}{k}"] = next(vals)
    F = np.zeros((3, 3))
    idx = np.array([1, 2, 3])
    for k, s in ((1, [1, 2]), (2, [1, 3])):
        Uk = np.array([[sym[f"a{k}"], sym[f"b{k}"]], [sym[f"c{k}"], sym[f"d{k}"]]])
        odense.extend_add(idx, np.array(s), Uk, F)
    expect = np.array([[sum(sym[t] for t in e.split("+")) if e != "0" else 0.0 for e in row]
                       for row in _rows("extend_add_example.txt")])
    assert np.array_equal(F, expect)


def test_extend_merge_fig2():
    """Eq. Rmerge / Fig. 2: the parent's R reuses the children's entries on
    shared rows and columns; keyed generation reproduces that provenance."""
    seed = 11
    Rg = lambda rows, d: orng.gaussian(seed, np.array(rows), d)
    R1 = Rg([1, 4, 5], 1)
    R2 = Rg([2, 3, 4, 5, 7], 2)
    R3 = Rg([4, 5, 6, 7], 3)
    src = {1: ({1: 0, 4: 1, 5: 2}, R1), 2: ({2: 0, 3: 1, 4: 2, 5: 3, 7: 4}, R2)}
    pos3 = {4: 0, 5: 1, 6: 2, 7: 3}
    for row, col, where in _rows("extend_merge_fig2.txt"):
        row, col = int(row), int(col) - 1
        val = R3[pos3[row], col]
        owners = [k for k in (1, 2) if row in src[k][0] and col < src[k][1].shape[1]]
        expect = {"1": [1], "2": [2], "12": [1, 2], "g": []}[where]
        assert owners == expect, (row, col)
        for k in owners:
            assert src[k][1][src[k][0][row], col] == val


def test_hss_tree_partition():
    nodes, k, q = osym.hss_tree(100, 37, 16)
    root = len(nodes) - 1
    assert nodes[root].children == [k, q]
    assert (nodes[k].lo, nodes[k].hi, nodes[q].lo, nodes[q].hi) == (0, 100, 100, 137)
    leaves = [nd for nd in nodes if nd.leaf]
    assert all(nd.m <= 16 for nd in leaves)
    assert sum(nd.m for nd in leaves) == 137
    for t, nd in enumerate(nodes):
        for c in nd.children:
            assert c < t        # postorder
        if nd.children:
            a, b = nd.children
            assert nodes[a].lo == nd.lo and nodes[a].hi == nodes[b].lo and nodes[b].hi == nd.hi
            if t != root:
                assert nodes[a].m == (nd.m + 1) // 2


def test_fv_assembly_values_and_their_gradient():
    """The differentiable finite-volume assembly reproduces the CSR values of
    fv_diffusion3d exactly, and its automatic derivative with respect to one
    kappa matches a central difference of the assembled values."""
    torch = pytest.importorskip("torch")
    n = 5
    kap, _ = P.smoothed_log_kappa(n, seed=3)
    A = P.fv_diffusion3d(n, kap)
    kt = torch.tensor(kap, requires_grad=True)
    v = P.fv_diffusion3d_values(n, kt)
    assert np.array_equal(v.detach().numpy(), A.val)
    w = np.random.default_rng(0).standard_normal(len(A.val))
    (v * torch.tensor(w)).sum().backward()
    c, h = 62, 1e-6
    kp, km = kap.copy(), kap.copy()
    kp[c] += h
    km[c] -= h
    fd = (P.fv_diffusion3d(n, kp).val - P.fv_diffusion3d(n, km).val) @ w / (2 * h)
    assert abs(kt.grad[c].item() - fd) <= 1e-7 * max(1.0, abs(fd))


def test_convdiff_batch_recipe():
    """The 256-system convection-diffusion batch: sides in [48, 160], speeds
    in [0, 20], total unknowns 3,100,693 and 140,346 fronts with 8^2 leaves;
    every system is its own elimination tree (one root)."""
    systems = P.convdiff_batch()
    assert len(systems) == 256
    sides = [int(round(np.sqrt(A.n))) for A, _, _ in systems]
    assert min(sides) >= 48 and max(sides) <= 160
    assert sum(A.n for A, _, _ in systems) == 3100693
    assert sum(len(o.parent) for _, o, _ in systems) == 140346
    for A, o, b in systems[:8]:
        assert int((o.parent == -1).sum()) == 1 and b.shape == (A.n,)


@pytest.mark.parametrize("ndim,n", [(2, 23), (3, 9)])
def test_paper_convection_diffusion_is_exact_on_linear_functions(ndim, n):
    """C2D / C3D (Sec. 6.1): first-order upwind differences are exact on
    linear functions, and the Laplacian vanishes on them, so at every point
    whose neighbours are all interior, (A u)/h^2 = v_a for u = the a-th
    coordinate; the matrix is a (weakly) diagonally dominant M-matrix."""
    A = P.convdiff_paper(n, ndim)
    S = A.to_scipy()
    h = 1.0 / (n + 1)
    N = n ** ndim
    idx = np.arange(N)
    coords, rem = [], idx.copy()
    for _ in range(ndim):
        coords.append(rem % n)
        rem = rem // n
    inner = np.all([(c > 0) & (c < n - 1) for c in coords], axis=0)
    x = [(c + 1) * h for c in coords]
    if ndim == 2:
        v = [x[0] * (1 - x[0]) * (2 * x[1] - 1), x[1] * (1 - x[1]) * (2 * x[0] - 1)]
    else:
        v = [2 * x[0] * (1 - x[0]) * (2 * x[1] - 1) * x[2], -x[1] * (1 - x[1]) * (2 * x[0] - 1),
             -(2 * x[0] - 1) * (2 * x[1] - 1) * x[2] * (1 - x[2])]
    for a in range(ndim):
        Au = S @ x[a] / h ** 2
        assert np.allclose(Au[inner], v[a][inner], rtol=0, atol=1e-9)
    import scipy.sparse as sp
    D = S.diagonal()
    C = S.tocoo()
    assert np.all(C.data[C.row != C.col] <= 0) and np.all(D > 0)
    assert np.all(D + np.asarray((S - sp.diags(D)).sum(axis=1)).ravel() >= -1e-15)
    assert abs(S - S.T).max() > 0   # not symmetric
