"""HSS toolkit (oracle side, FP64): interpolative decomposition, randomized
compression (Alg. 1) with the adaptive-rank loop, HSS matvec and element
extraction, ULV-like factorization and solves, low-rank Schur product.

Notation follows Sec. 2 of the paper.  Per node tau of a postordered binary
tree: row generator U_tau = Pi^r [I; E^r] (m_r x r), column generator
V_tau = Pi^c [I; E^c] (m_c x c) (Eq. UVstructure), D_tau at leaves, B_{nu1,nu2}
and B_{nu2,nu1} stored at the parent (Sec. 2.1).  A permutation is stored as
an index array ``perm`` with (Pi^T x)[i] = x[perm[i]], so U[perm[:r]] = I and
U[perm[r:]] = E.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .symbolic import hss_tree


class RankError(RuntimeError):
    """Adaptive sampling reached d_max without every ID succeeding."""


# ---------------------------------------------------------------------------
# interpolative decomposition (Sec. 2.2, Eq. for ID; stopping rule Sec. 5.3)
# ---------------------------------------------------------------------------

def _householder_step(W, perm, j, p, nrm):
    """Step j of a column-pivoted Householder QR of W in place: interchange
    positions j and p (columns of W and entries of perm), then reduce column
    j below row j with the reflector of its remaining norm nrm, applied to
    columns j.. ."""
    if p != j:
        W[:, [j, p]] = W[:, [p, j]]
        perm[[j, p]] = perm[[p, j]]
    x = W[j:, j]
    alpha = -np.copysign(nrm, x[0]) if x[0] != 0 else -nrm
    v = x.copy()
    v[0] -= alpha
    vn = np.dot(v, v)
    if vn > 0:
        W[j:, j:] -= np.outer(v, (2.0 / vn) * (v @ W[j:, j:]))
    W[j, j] = alpha
    W[j + 1:, j] = 0.0


def cpqr_eps(Y, eps, atol=0.0):
    """Householder QR with column pivoting of Y (d x m), stopped at the
    numerical rank.  At every step the pivot is the column whose remaining
    part has the largest 2-norm, recomputed from the updated column (ties go
    to the lowest index).  The factorization stops before step i+1 when that
    norm is <= eps times the first pivot's norm, i.e. |R_{i+1,i+1}| <= eps
    |R_11| (the modified geqp3 of Sec. 5.3), or <= the absolute tolerance
    atol (0: the relative rule alone).  It stops before the first step when
    the largest column norm is <= atol, so a zero matrix has rank 0.

    Returns (perm, R, k): Y[:, perm] = Q R with R (min(d,m) x m) upper
    trapezoidal in its first k rows; only R[:k] is meaningful."""
    W = np.array(Y, dtype=np.float64, copy=True)
    d, m = W.shape
    perm = np.arange(m)
    kmax = min(d, m)
    first = None
    k = 0
    for j in range(kmax):
        norms = np.sqrt(np.sum(W[j:, j:] ** 2, axis=0))
        p = j + int(np.argmax(norms))
        nrm = norms[p - j]
        if first is None:
            first = nrm
            if first <= atol:
                break
        elif nrm <= max(eps * first, atol):
            break
        _householder_step(W, perm, j, p, nrm)
        k = j + 1
    return perm, W[:kmax], k


def qr_forced(Y, order):
    """Householder QR of Y (d x m) whose pivots are the columns ``order``
    (original indices), taken in that sequence, with the interchange
    bookkeeping of cpqr_eps.  Returns (perm, W): Y[:, perm] = Q W with W
    (d x m) upper triangular in its first k = len(order) columns; rows < k
    of the other columns hold R12, rows >= k hold R22."""
    W = np.array(Y, dtype=np.float64, copy=True)
    m = W.shape[1]
    perm = np.arange(m)
    for j, c in enumerate(order):
        p = int(np.flatnonzero(perm == c)[0])
        nrm = np.sqrt(np.sum(W[j:, p] ** 2))
        _householder_step(W, perm, j, p, nrm)
    return perm, W


SRRQR_MAX_SWAPS = 64


def strong_rrqr(Y, perm, k, f, max_swaps=SRRQR_MAX_SWAPS):
    """Strong rank-revealing QR with the rank k held fixed (Gu and
    Eisenstat, SIAM J. Sci. Comput. 17 (1996), the algorithm for a given k),
    started from the selection perm[:k] of a column-pivoted QR; Sec. 2.2 and
    Sec. 7 name it as a replacement of that QR inside the ID.

    With Y[:, perm] = Q [R11 R12; 0 R22], interchanging selected column i
    with remaining column j multiplies |det R11| by sqrt(rho_ij), where
    rho_ij = (R11^{-1} R12)_ij^2 + gamma_j^2 / omega_i^2, gamma_j the
    2-norm of column j of R22 and 1/omega_i the 2-norm of row i of
    R11^{-1}.  While the largest rho (ties: lowest i + k j) exceeds f^2,
    column i leaves the selection, column j joins it as the last selected
    column, and Y is factored again in that pivot order.  At the end every
    |(R11^{-1} R12)_ij| <= f, unless max_swaps interchanges were made first.

    Returns (perm, W, swaps) with W as from qr_forced."""
    m = Y.shape[1]
    order = [int(c) for c in perm[:k]]
    swaps = 0
    while True:
        perm, W = qr_forced(Y, order)
        if k == 0 or k == m:
            return perm, W, swaps
        R11 = W[:k, :k]
        X = sla.solve_triangular(R11, W[:k, k:], lower=False)
        Z = sla.solve_triangular(R11, np.eye(k), lower=False)
        gam2 = np.sum(W[k:, k:] ** 2, axis=0)
        rho = X ** 2 + np.outer(np.sum(Z ** 2, axis=1), gam2)
        e = int(np.argmax(rho.ravel(order="F")))
        i, j = e % k, e // k
        if not rho[i, j] > f * f or swaps >= max_swaps:
            return perm, W, swaps
        order = [int(perm[t]) for t in range(k) if t != i] + [int(perm[k + j])]
        swaps += 1


def interp_decomp(Y, eps, atol=0.0, srrqr_f=0.0, stats=None):
    """[X, J] = ID(Y, eps): Y ~= Y[:, J] X with X = [I, R1^{-1} R2] Pi^{-1}
    (Sec. 2.2).  Returns (perm, E, k) where J = perm[:k] and
    E = (R1^{-1} R2)^T, so that Y^T ~= Pi [I; E] Y[:, J]^T.  The rank k comes
    from cpqr_eps; with srrqr_f > 0 the selection is then improved by
    strong_rrqr with f = srrqr_f (k unchanged), and stats["swaps"] (when a
    dict is given) counts its interchanges."""
    perm, R, k = cpqr_eps(Y, eps, atol)
    m = Y.shape[1]
    if k == 0:
        return perm, np.zeros((m, 0)), 0
    if srrqr_f > 0 and k < m:
        perm, R, sw = strong_rrqr(Y, perm, k, srrqr_f)
        if stats is not None:
            stats["swaps"] = stats.get("swaps", 0) + sw
    X = sla.solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    return perm, X.T.copy(), k


def interp_matrix(perm, E):
    """Dense Pi [I; E] (m x k)."""
    m = len(perm)
    k = E.shape[1]
    U = np.zeros((m, k))
    U[perm[:k]] = np.eye(k)
    U[perm[k:]] = E
    return U


# ---------------------------------------------------------------------------
# HSS data
# ---------------------------------------------------------------------------

@dataclass
class NodeGen:
    D: np.ndarray = None        # leaf diagonal block
    B12: np.ndarray = None      # at a parent: B_{nu1,nu2}
    B21: np.ndarray = None      # at a parent: B_{nu2,nu1}
    Uperm: np.ndarray = None
    UE: np.ndarray = None
    Vperm: np.ndarray = None
    VE: np.ndarray = None
    Ir: np.ndarray = None       # skeleton rows (local indices of the HSS matrix)
    Ic: np.ndarray = None       # skeleton columns

    @property
    def r(self):
        return self.UE.shape[1]

    @property
    def c(self):
        return self.VE.shape[1]

    def U(self):
        return interp_matrix(self.Uperm, self.UE)

    def V(self):
        return interp_matrix(self.Vperm, self.VE)


@dataclass
class HSS:
    """An HSS matrix on the node ranges of ``nodes`` (postorder)."""
    nodes: list
    gen: list
    root: int
    stats: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# randomized compression (Alg. 1) with adaptive rank (Sec. 2.2.1, Sec. 4.3)
# ---------------------------------------------------------------------------

def power_samples(op, R, q):
    """Samples of F and F^T with q steps of power iteration (Sec. 2.2, the
    power-iteration variant the paper describes and leaves as an option):
    S^r = (F F^T)^q F R and S^c = (F^T F)^q F^T R, with the matrices Alg. 1
    then takes in place of R: R^r = F^T (F F^T)^(q-1) F R for the row side
    (S^r = F R^r) and R^c = F (F^T F)^(q-1) F^T R for the column side
    (S^c = F^T R^c).  q = 0 is the plain sampling, R^r = R^c = R.  No
    reorthogonalization between the products (the paper names it as a
    possible need, without making it part of the scheme)."""
    Sr, Sc = op.sample(R)
    Rr = Rc = R
    for _ in range(q):
        Rr = op.sample(Sr)[1]    # F^T applied to the current row samples
        Rc = op.sample(Sc)[0]    # F applied to the current column samples
        Sr = op.sample(Rr)[0]
        Sc = op.sample(Rc)[1]
    return Sr, Sc, Rr, Rc


def compress(op, nodes, root, rand, eps, d0, dd, p, d_max, atol=0.0, power_q=0, srrqr_f=0.0):
    """Alg. 1 applied to a matrix known through ``op``:
    op.sample(R) -> (F R, F^T R) for a block of random columns and
    op.extract(I, J) -> F[I][:, J].  ``rand(c0, nc)`` returns columns
    [c0, c0+nc) of the random matrix R (n x nc).  With power_q > 0 the
    samples come from ``power_samples``, and the row side of every node
    takes R^r, the column side R^c, where plain sampling takes R for both.

    Bottom-up over the tree.  Reading of the paper's ID failure test (not
    stated there): a node succeeds iff its rank k satisfies k <= d - p or
    k == (rows of S_tau).  If a node fails, d grows by dd; nodes that
    succeeded keep their ID, D and B and only compute the new columns of
    their reduced samples and random matrices (Sec. 2.2.1); failed nodes are
    recomputed on all d columns."""
    nn = len(nodes)
    gen = [NodeGen() for _ in range(nn)]
    done = [False] * nn
    Sr_red = [None] * nn
    Sc_red = [None] * nn
    Rr_red = [None] * nn
    Rc_red = [None] * nn
    d = d0
    Sr, Sc, Rr, Rc = power_samples(op, rand(0, d), power_q)
    rounds = 0
    # record of the work done, for the algorithmic operation counts only
    # (oracle.work): columns sampled per pass, and per ID attempt the node,
    # side, samples d, rows m and rank k
    log = dict(sampled=[d], ids=[], node_cols=[])
    swaps = {}   # strong-RRQR interchanges of the IDs kept (nodes that succeeded)

    def node_samples(t, cols):
        """Unreduced S^r_tau, S^c_tau on columns ``cols`` (Alg. 1, leaf and
        non-leaf sample updates)."""
        nd = nodes[t]
        g = gen[t]
        if nd.leaf:
            I = np.arange(nd.lo, nd.hi)
            return Sr[I][:, cols] - g.D @ Rr[I][:, cols], Sc[I][:, cols] - g.D.T @ Rc[I][:, cols]
        a, b = nd.children
        sr = np.vstack([Sr_red[a][:, cols] - g.B12 @ Rr_red[b][:, cols],
                        Sr_red[b][:, cols] - g.B21 @ Rr_red[a][:, cols]])
        sc = np.vstack([Sc_red[a][:, cols] - g.B21.T @ Rc_red[b][:, cols],
                        Sc_red[b][:, cols] - g.B12.T @ Rc_red[a][:, cols]])
        return sr, sc

    def reduce_node(t, sr, sc, cols):
        """Row selection of the samples and the random-matrix update
        R^r_tau = V^T R, R^c_tau = U^T R (Alg. 1, lines after the ID)."""
        nd = nodes[t]
        g = gen[t]
        if nd.leaf:
            I = np.arange(nd.lo, nd.hi)
            Rr_in = Rr[I][:, cols]
            Rc_in = Rc[I][:, cols]
        else:
            a, b = nd.children
            Rr_in = np.vstack([Rr_red[a][:, cols], Rr_red[b][:, cols]])
            Rc_in = np.vstack([Rc_red[a][:, cols], Rc_red[b][:, cols]])
        return (sr[g.Uperm[:g.r]], sc[g.Vperm[:g.c]], g.V().T @ Rr_in, g.U().T @ Rc_in)

    while True:
        allc = np.arange(d)
        for t in range(nn):
            nd = nodes[t]
            if done[t] or any(not done[ch] for ch in nd.children):
                continue
            g = gen[t]
            if nd.leaf:
                I = np.arange(nd.lo, nd.hi)
                if g.D is None:
                    g.D = op.extract(I, I)
            else:
                a, b = nd.children
                g.B12 = op.extract(gen[a].Ir, gen[b].Ic)
                g.B21 = op.extract(gen[b].Ir, gen[a].Ic)
            if t == root:
                done[t] = True
                continue
            sr, sc = node_samples(t, allc)
            sw_node = {}
            pu, Eu, kr = interp_decomp(sr.T, eps, atol, srrqr_f, sw_node)
            pv, Ev, kc = interp_decomp(sc.T, eps, atol, srrqr_f, sw_node)
            log["ids"].append((t, d, sr.shape[0], kr, sc.shape[0], kc))
            ok_r = kr <= d - p or kr == sr.shape[0]
            ok_c = kc <= d - p or kc == sc.shape[0]
            if not (ok_r and ok_c):
                continue
            swaps["swaps"] = swaps.get("swaps", 0) + sw_node.get("swaps", 0)
            g.Uperm, g.UE, g.Vperm, g.VE = pu, Eu, pv, Ev
            if nd.leaf:
                base_r = base_c = np.arange(nd.lo, nd.hi)
            else:
                a, b = nd.children
                base_r = np.concatenate([gen[a].Ir, gen[b].Ir])
                base_c = np.concatenate([gen[a].Ic, gen[b].Ic])
            g.Ir = base_r[pu[:kr]]
            g.Ic = base_c[pv[:kc]]
            Sr_red[t], Sc_red[t], Rr_red[t], Rc_red[t] = reduce_node(t, sr, sc, allc)
            log["node_cols"].append((t, d))
            done[t] = True
        if done[root]:
            break
        if d + dd > d_max:
            raise RankError(f"HSS compression needs more than d_max={d_max} samples")
        Srn, Scn, Rrn, Rcn = power_samples(op, rand(d, dd), power_q)
        log["sampled"].append(dd)
        Rr = np.hstack([Rr, Rrn])
        Rc = np.hstack([Rc, Rcn])
        Sr = np.hstack([Sr, Srn])
        Sc = np.hstack([Sc, Scn])
        newc = np.arange(d, d + dd)
        d += dd
        rounds += 1
        for t in range(nn):
            if done[t] and t != root:
                sr, sc = node_samples(t, newc)
                a1, a2, a3, a4 = reduce_node(t, sr, sc, newc)
                log["node_cols"].append((t, dd))
                Sr_red[t] = np.hstack([Sr_red[t], a1])
                Sc_red[t] = np.hstack([Sc_red[t], a2])
                Rr_red[t] = np.hstack([Rr_red[t], a3])
                Rc_red[t] = np.hstack([Rc_red[t], a4])
    return HSS(nodes, gen, root, dict(d=d, rounds=rounds, log=log, swaps=swaps.get("swaps", 0)))


# ---------------------------------------------------------------------------
# HSS matvec, nested bases, extraction, expansion (Sec. 2.1, Sec. 4.5)
# ---------------------------------------------------------------------------

def _subtree(nodes, rt):
    out = []

    def rec(t):
        for c in nodes[t].children:
            rec(c)
        out.append(t)
    rec(rt)
    return out


def up_sweep(H, rt, X, which):
    """x_hat at every node of the subtree of ``rt`` (rt excluded):
    leaf x_hat = G^T X(I_tau), non-leaf x_hat = G^T [x_hat_1; x_hat_2], with
    G = U (which='U') or V.  X is indexed by the HSS matrix's local rows."""
    xh = {}
    for t in _subtree(H.nodes, rt):
        if t == rt:
            continue
        nd = H.nodes[t]
        G = H.gen[t].U() if which == "U" else H.gen[t].V()
        if nd.leaf:
            xh[t] = G.T @ X[nd.lo:nd.hi]
        else:
            a, b = nd.children
            xh[t] = G.T @ np.vstack([xh[a], xh[b]])
    return xh


def down_expand(H, rt, y, which):
    """G^big_rt y for G = U or V: expand a coefficient block through the
    nested bases of the subtree of rt (Eq. nestedUV).  Returns rows over the
    range of rt."""
    nd0 = H.nodes[rt]
    out = np.zeros((nd0.hi - nd0.lo, y.shape[1]))

    def rec(t, yt):
        nd = H.nodes[t]
        G = H.gen[t].U() if which == "U" else H.gen[t].V()
        v = G @ yt
        if nd.leaf:
            out[nd.lo - nd0.lo:nd.hi - nd0.lo] = v
        else:
            a, b = nd.children
            ra = H.gen[a].r if which == "U" else H.gen[a].c
            rec(a, v[:ra])
            rec(b, v[ra:])
    rec(rt, y)
    return out


def big_t(H, rt, X, which):
    """(G^big_rt)^T X for G = U or V, X with rows over rt's range:
    leaf G^T X(I_tau), non-leaf G^T [child results] (Eq. nestedUV)."""
    nd = H.nodes[rt]
    lo0 = nd.lo

    def rec(t):
        n = H.nodes[t]
        G = H.gen[t].U() if which == "U" else H.gen[t].V()
        if n.leaf:
            return G.T @ X[n.lo - lo0:n.hi - lo0]
        a, b = n.children
        return G.T @ np.vstack([rec(a), rec(b)])
    return rec(rt)


def hss_matvec(H, rt, X, trans=False):
    """Y = F X (or F^T X) for the HSS submatrix on the subtree of ``rt``:
    up-sweep with V^T (U^T), sibling products with B, down-sweep with U (V),
    diagonal blocks at the leaves.  X rows are local to rt's range."""
    nodes, gen = H.nodes, H.gen
    lo0 = nodes[rt].lo
    X = X.reshape(X.shape[0], -1)
    Xl = np.zeros((nodes[rt].hi, X.shape[1]))
    Xl[lo0:] = X
    xh = up_sweep(H, rt, Xl, "U" if trans else "V")
    yh = {}
    order = _subtree(nodes, rt)
    for t in order:
        nd = nodes[t]
        if nd.leaf:
            continue
        a, b = nd.children
        g = gen[t]
        if not trans:
            yh[a] = g.B12 @ xh[b]
            yh[b] = g.B21 @ xh[a]
        else:
            yh[a] = g.B21.T @ xh[b]
            yh[b] = g.B12.T @ xh[a]
    Y = np.zeros_like(X)
    for t in reversed(order):           # preorder: parents before children
        nd = nodes[t]
        g = gen[t]
        if t != rt and not nd.leaf:
            G = g.V() if trans else g.U()
            v = G @ yh[t]
            a, b = nd.children
            ra = (gen[a].c if trans else gen[a].r)
            yh[a] = yh[a] + v[:ra]
            yh[b] = yh[b] + v[ra:]
        if nd.leaf:
            Dt = g.D.T if trans else g.D
            y = Dt @ Xl[nd.lo:nd.hi]
            if t != rt:
                G = g.V() if trans else g.U()
                y = y + G @ yh[t]
            Y[nd.lo - lo0:nd.hi - lo0] = y
    return Y


def hss_extract(H, rt, I, J):
    """Entries F[I][:, J] of the HSS submatrix on rt (local indices): the
    paper's extraction by multiplication with unit vectors (Sec. 4.5)."""
    n = H.nodes[rt].hi - H.nodes[rt].lo
    E = np.zeros((n, len(J)))
    E[np.asarray(J), np.arange(len(J))] = 1.0
    return hss_matvec(H, rt, E)[np.asarray(I)]


def hss_dense(H, rt):
    """Dense expansion of the HSS submatrix on rt (Eq. HSSexamplematrix):
    D at the leaves, U^big_1 B_12 (V^big_2)^T for every sibling pair."""
    nodes, gen = H.nodes, H.gen
    lo0 = nodes[rt].lo
    n = nodes[rt].hi - lo0
    F = np.zeros((n, n))
    for t in _subtree(nodes, rt):
        nd = nodes[t]
        if nd.leaf:
            F[nd.lo - lo0:nd.hi - lo0, nd.lo - lo0:nd.hi - lo0] = gen[t].D
        else:
            a, b = nd.children
            na, nb = nodes[a], nodes[b]
            Ua = down_expand(H, a, np.eye(gen[a].r), "U")
            Ub = down_expand(H, b, np.eye(gen[b].r), "U")
            Va = down_expand(H, a, np.eye(gen[a].c), "V")
            Vb = down_expand(H, b, np.eye(gen[b].c), "V")
            F[na.lo - lo0:na.hi - lo0, nb.lo - lo0:nb.hi - lo0] = Ua @ gen[t].B12 @ Vb.T
            F[nb.lo - lo0:nb.hi - lo0, na.lo - lo0:na.hi - lo0] = Ub @ gen[t].B21 @ Va.T
    return F


# ---------------------------------------------------------------------------
# ULV-like factorization (Sec. 2.3) of the subtree rooted at k
# ---------------------------------------------------------------------------

@dataclass
class ULVNode:
    perm: np.ndarray = None   # Pi^r of the row generator
    E: np.ndarray = None
    L: np.ndarray = None      # (m-r) x (m-r) lower triangular
    Q: np.ndarray = None      # m x m orthogonal, W[:m-r] = [L 0] Q^T ... stored as Qt (see below)
    D21: np.ndarray = None    # r x (m-r)
    V1: np.ndarray = None     # (m-r) x c
    m: int = 0
    r: int = 0


@dataclass
class ULV:
    H: HSS
    k: int
    nodes: dict               # node id -> ULVNode (nodes of k's subtree except k)
    lu: tuple = None          # scipy lu_factor of D~_k
    Vbar_k: np.ndarray = None  # diag(V^_1, V^_2) V_k (or V_k at a leaf); None if k has no generator


def ulv_factor(H, k):
    """ULV-like factorization of the HSS submatrix on the subtree of k.

    Reconstructed from the paper's description (Sec. 2.3: Omega_tau with
    Omega_tau U_tau = [0; I], then an LQ step, merging up the tree, LU at the
    top node) and the low-rank Schur formula of Sec. 4.4.  For every node tau
    of the subtree other than k, in postorder:
      Dbar = D_tau (leaf) or [D^_1, B12 V^_2^T; B21 V^_1^T, D^_2];
      Vbar = V_tau (leaf) or diag(V^_1, V^_2) V_tau;
      W = Omega_tau Dbar, Omega_tau = [-E I; I 0] Pi^T;
      W[:m-r] = [L 0] Q (LQ);  W Q^T = [L 0; D^21 D^];  Q Vbar = [V^1; V^].
    At k: Dtilde_k = merged block, P L U = Dtilde_k (partial pivoting).
    Pinned by the dense identity: ULV solves equal dense LU solves with the
    expanded HSS matrix."""
    nodes, gen = H.nodes, H.gen
    out = {}
    Dhat = {}
    Vhat = {}

    def merged(t):
        nd = nodes[t]
        g = gen[t]
        if nd.leaf:
            return g.D.copy(), (g.V() if g.VE is not None else None)
        a, b = nd.children
        Db = np.block([[Dhat[a], g.B12 @ Vhat[b].T], [g.B21 @ Vhat[a].T, Dhat[b]]])
        Vb = None
        if g.VE is not None:
            ca = Vhat[a].shape[1]
            V = g.V()
            Vb = np.vstack([Vhat[a] @ V[:ca], Vhat[b] @ V[ca:]])
        return Db, Vb

    for t in _subtree(nodes, k):
        if t == k:
            continue
        g = gen[t]
        Db, Vb = merged(t)
        m = Db.shape[0]
        r = g.r
        perm, E = g.Uperm, g.UE
        P = Db[perm]
        W = np.vstack([P[r:] - E @ P[:r], P[:r]])
        nl = m - r
        if nl > 0:
            Qf, Rf = np.linalg.qr(W[:nl].T, mode="complete")   # W1^T = Qf [R1; 0]
            L = Rf[:nl].T
        else:
            Qf = np.eye(m)
            L = np.zeros((0, 0))
        WQ = W[nl:] @ Qf
        QV = Qf.T @ Vb
        out[t] = ULVNode(perm, E, L, Qf, WQ[:, :nl], QV[:nl], m, r)
        Dhat[t] = WQ[:, nl:]
        Vhat[t] = QV[nl:]
    Dk, Vbk = merged(k)
    return ULV(H, k, out, sla.lu_factor(Dk), Vbk)


def ulv_solve(F, b):
    """Solve Ftilde_k z = b (rows local to k's range) with the ULV factors:
    up-sweep (Omega, L^{-1}, reduced right-hand sides and the known coupling
    terms w), LU solve at k, down-sweep applying Q^T."""
    H, k = F.H, F.k
    nodes, gen = H.nodes, H.gen
    lo0 = nodes[k].lo
    b = b.reshape(b.shape[0], -1)
    chat, w, y1 = {}, {}, {}

    def rhs(t):
        nd = nodes[t]
        if nd.leaf:
            return b[nd.lo - lo0:nd.hi - lo0]
        a, c = nd.children
        g = gen[t]
        return np.vstack([chat[a] - g.B12 @ w[c], chat[c] - g.B21 @ w[a]])

    for t in _subtree(nodes, k):
        if t == k:
            continue
        u = F.nodes[t]
        bb = rhs(t)
        P = bb[u.perm]
        cvec = np.vstack([P[u.r:] - u.E @ P[:u.r], P[:u.r]])
        nl = u.m - u.r
        y = sla.solve_triangular(u.L, cvec[:nl], lower=True) if nl else np.zeros((0, b.shape[1]))
        y1[t] = y
        chat[t] = cvec[nl:] - u.D21 @ y
        wt = u.V1.T @ y
        if not nodes[t].leaf:
            a, c = nodes[t].children
            wt = wt + gen[t].V().T @ np.vstack([w[a], w[c]])
        w[t] = wt
    yk = sla.lu_solve(F.lu, rhs(k))
    z = np.zeros((nodes[k].hi - lo0, b.shape[1]))

    def down(t, y2):
        nd = nodes[t]
        if t == k:
            xb = y2
        else:
            u = F.nodes[t]
            xb = u.Q @ np.vstack([y1[t], y2])
        if nd.leaf:
            z[nd.lo - lo0:nd.hi - lo0] = xb
        else:
            a, c = nd.children
            ra = xb.shape[0] - F.nodes[c].r
            down(a, xb[:ra])
            down(c, xb[ra:])
    down(k, yk)
    return z


def ulv_solve_transpose(F, g_in):
    """Solve Ftilde_k^T lam = g with the same factors.  With the transformed
    unknowns lam_tau = Omega_tau^T [mu1; mu2] the system is block upper
    triangular: up-sweep applies Q to the right-hand side and passes its
    bottom part up, the top node solves Dtilde_k^T, and the down-sweep
    recovers mu1 = L^{-T}(g~1 - D^21^T mu2 - V^1 h), where h carries the
    off-diagonal coupling B^T mu2 of the sibling and V of the parent."""
    H, k = F.H, F.k
    nodes, gen = H.nodes, H.gen
    lo0 = nodes[k].lo
    g_in = g_in.reshape(g_in.shape[0], -1)
    nr = g_in.shape[1]
    gt1, gt2 = {}, {}

    def rhs(t):
        nd = nodes[t]
        if nd.leaf:
            return g_in[nd.lo - lo0:nd.hi - lo0]
        a, c = nd.children
        return np.vstack([gt2[a], gt2[c]])

    for t in _subtree(nodes, k):
        if t == k:
            continue
        u = F.nodes[t]
        gg = u.Q.T @ rhs(t)
        nl = u.m - u.r
        gt1[t] = gg[:nl]
        gt2[t] = gg[nl:]
    lam_k = sla.lu_solve(F.lu, rhs(k), trans=1)
    lam = np.zeros((nodes[k].hi - lo0, nr))

    def down(t, lbar, h):
        nd = nodes[t]
        if nd.leaf:
            lam[nd.lo - lo0:nd.hi - lo0] = lbar
            return
        a, c = nd.children
        g = gen[t]
        ra = F.nodes[a].r
        mu_a, mu_c = lbar[:ra], lbar[ra:]
        ha = g.B21.T @ mu_c
        hc = g.B12.T @ mu_a
        if h is not None:
            V = g.V()
            ca = gen[a].c
            ha = ha + V[:ca] @ h
            hc = hc + V[ca:] @ h
        for ch, mu2, hh in ((a, mu_a, ha), (c, mu_c, hc)):
            u = F.nodes[ch]
            nl = u.m - u.r
            if nl:
                rhs1 = gt1[ch] - u.D21.T @ mu2 - u.V1 @ hh
                mu1 = sla.solve_triangular(u.L, rhs1, lower=True, trans=1)
            else:
                mu1 = np.zeros((0, nr))
            lb = np.zeros((u.m, nr))
            lb[u.perm[:u.r]] = mu2 - u.E.T @ mu1
            lb[u.perm[u.r:]] = mu1
            down(ch, lb, hh)
    down(k, lam_k, None)
    return lam


def schur_lowrank(F, q):
    """Theta^* and Phi of the low-rank Schur product
    F21 F11^{-1} F12 = Theta^* Phi (Sec. 4.4) for a front whose HSS root has
    children k (F11) and q (F22):
      Theta^* = U^big_q B_qk Vbar_k^T U_LU^{-1},
      Phi     = L_LU^{-1} P^T U_k B_kq (V^big_q)^T,
    with P L U = Dtilde_k from the ULV factorization.  The paper prints this
    formula only in a commented-out, partly garbled form; this is our reading,
    pinned by the dense identity Theta^* Phi = F21 F11^{-1} F12."""
    H = F.H
    k = F.k
    root = H.nodes[k].parent
    g = H.gen[root]
    gk = H.gen[k]
    lu, piv = F.lu
    m = lu.shape[0]
    P = np.eye(m)
    for i, pv in enumerate(piv):       # row interchanges of getrf
        P[[i, pv]] = P[[pv, i]]
    # P_rows D = L U  with P_rows built from the interchanges; D = P_rows^T L U
    Lf = np.tril(lu, -1) + np.eye(m)
    Uf = np.triu(lu)
    Ubig_q = down_expand(H, q, np.eye(H.gen[q].r), "U")
    Vbig_q = down_expand(H, q, np.eye(H.gen[q].c), "V")
    B_qk = g.B21 if H.nodes[root].children[0] == k else g.B12
    B_kq = g.B12 if H.nodes[root].children[0] == k else g.B21
    T = (Ubig_q @ B_qk) @ F.Vbar_k.T
    Theta = sla.solve_triangular(Uf, T.T, lower=False, trans=1).T
    Phi = sla.solve_triangular(Lf, P @ (gk.U() @ (B_kq @ Vbig_q.T)), lower=True, unit_diagonal=True)
    return Theta, Phi


class Front11Ops:
    """Products with the off-diagonal blocks of an HSS front (Sec. 4.4):
    F21 = U^big_q B_qk (V^big_k)^T and F12 = U^big_k B_kq (V^big_q)^T."""

    def __init__(self, H, k, q):
        self.H, self.k, self.q = H, k, q
        root = H.nodes[k].parent
        g = H.gen[root]
        self.B_kq, self.B_qk = g.B12, g.B21   # k is the first child by construction

    def _vt(self, rt, x, which):
        return big_t(self.H, rt, x, which)

    def f21(self, z):
        return down_expand(self.H, self.q, self.B_qk @ self._vt(self.k, z, "V"), "U")

    def f12(self, x):
        return down_expand(self.H, self.k, self.B_kq @ self._vt(self.q, x, "V"), "U")

    def f12t(self, z):
        return down_expand(self.H, self.q, self.B_kq.T @ self._vt(self.k, z, "U"), "V")

    def f21t(self, x):
        return down_expand(self.H, self.k, self.B_qk.T @ self._vt(self.q, x, "U"), "V")


def build_hss_front(op, s, u, leaf_size, rand, eps, d0, dd, p, d_max, atol=0.0, power_q=0, srrqr_f=0.0):
    """Compress a front of size s+u (Alg. 1), then ULV-factor its F11 part and
    form Theta^*, Phi.  Returns (H, ULV, k, q, Theta, Phi)."""
    nodes, k, q = hss_tree(s, u, leaf_size)
    root = len(nodes) - 1
    H = compress(op, nodes, root, rand, eps, d0, dd, p, d_max, atol, power_q, srrqr_f)
    F = ulv_factor(H, k)
    Theta = Phi = None
    if q >= 0:
        Theta, Phi = schur_lowrank(F, q)
    return H, F, k, q, Theta, Phi
