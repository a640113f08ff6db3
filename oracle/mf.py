"""Multifrontal factorization with dense and HSS fronts (oracle side, FP64).

Sec. 3 (multifrontal LU, extend-add, forward/backward solve) and Sec. 4
(HSS fronts: random sampling with skinny extend-add, Alg. 1, ULV, low-rank
Schur update) of the paper.

Reading of the front-selection rule: a front is HSS iff its separator has at
least ``min_sep_hss`` indices (the paper selects whole etree levels above a
switch level; a separator-size threshold plays that role on the graded
separator sizes of nested dissection).
"""
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import dense as dn
from . import hss as hs
from .rng import gaussian
from .symbolic import analyse, permute_csr


@dataclass
class Options:
    min_sep_hss: int = 1 << 30
    leaf_size: int = 64
    rel_tol: float = 1e-6
    d0: int = 128
    dd: int = 128
    p: int = 10
    d_max: int = 1 << 20
    seed: int = 0
    abs_tol: float = 0.0
    power_q: int = 0   # steps of power iteration in the sampling (0: plain sampling)
    srrqr_f: float = 0.0   # strong-RRQR bound f inside the IDs (0: column-pivoted QR alone)


class DenseUpdate:
    def __init__(self, M):
        self.M = M

    def matvec(self, X):
        return self.M @ X

    def rmatvec(self, X):
        return self.M.T @ X

    def extract(self, I, J):
        return self.M[np.ix_(I, J)]

    def dense(self):
        return self.M


class HSSUpdate:
    """U = F22 - Theta^* Phi with F22 the HSS subtree q of a child front
    (Sec. 4.4): products by HSS matvec plus two dense products, entries by
    extraction minus the low-rank term."""

    def __init__(self, H, q, Theta, Phi):
        self.H, self.q, self.Theta, self.Phi = H, q, Theta, Phi

    def matvec(self, X):
        return hs.hss_matvec(self.H, self.q, X) - self.Theta @ (self.Phi @ X)

    def rmatvec(self, X):
        return hs.hss_matvec(self.H, self.q, X, trans=True) - self.Phi.T @ (self.Theta.T @ X)

    def extract(self, I, J):
        I = np.asarray(I, dtype=np.int64)
        J = np.asarray(J, dtype=np.int64)
        if len(I) == 0 or len(J) == 0:
            return np.zeros((len(I), len(J)))
        return hs.hss_extract(self.H, self.q, I, J) - self.Theta[I] @ self.Phi[:, J]

    def dense(self):
        u = self.Theta.shape[0]
        return self.matvec(np.eye(u))


class FrontOp:
    """The frontal matrix F_i = A_i (+) U_nu1 (+) U_nu2 (Eq. frontal_1), known
    only through products with random blocks (Eq. FtimesR: A_i R plus the
    row-extended children's products, Sec. 4.3) and entry extraction (Sec. 4.5)."""

    def __init__(self, Ap, front, fronts, updates):
        idx = front.idx
        s = front.s
        sub = Ap[idx][:, idx].tocoo()
        keep = (sub.row < s) | (sub.col < s)
        import scipy.sparse as sp
        self.Ai = sp.csr_matrix((sub.data[keep], (sub.row[keep], sub.col[keep])), shape=sub.shape)
        self.n = len(idx)
        self.kids = []
        for c in front.children:
            pos = np.searchsorted(idx, fronts[c].upd)
            assert np.all(idx[pos] == fronts[c].upd)
            self.kids.append((pos, updates[c]))

    def sample(self, R):
        Sr = self.Ai @ R
        Sc = self.Ai.T @ R
        for pos, Uc in self.kids:
            Rc = R[pos]
            Sr[pos] += Uc.matvec(Rc)
            Sc[pos] += Uc.rmatvec(Rc)
        return Sr, Sc

    def extract(self, I, J):
        I = np.asarray(I, dtype=np.int64)
        J = np.asarray(J, dtype=np.int64)
        out = self.Ai[I][:, J].toarray()
        for pos, Uc in self.kids:
            inv = -np.ones(self.n, dtype=np.int64)
            inv[pos] = np.arange(len(pos))
            ii = np.nonzero(inv[I] >= 0)[0]
            jj = np.nonzero(inv[J] >= 0)[0]
            if len(ii) and len(jj):
                out[np.ix_(ii, jj)] += Uc.extract(inv[I][ii], inv[J][jj])
        return out


@dataclass
class FrontFactor:
    kind: str
    data: dict


@dataclass
class Factorization:
    n: int
    perm: np.ndarray
    Ap: object
    fronts: list
    factors: list
    opts: Options


def factor(A, ordering, opts, stop_after=None, record=None):
    """Numeric multifrontal factorization, fronts in postorder (Sec. 3.2).
    ``stop_after`` ends the loop after that front id (a bounded sample of the
    work for timing; the result is then not a usable factorization).
    Dense fronts: assembly, extend-add, partial LU.  HSS fronts: random
    matrix keyed by original row id, samples by skinny extend-add, Alg. 1
    with adaptive rank, ULV of F11 and Theta^*, Phi (Sec. 4).
    ``record``: None, or a dict that receives, per HSS front id, the front
    operator, its random-matrix function, the HSS generators, Theta^*, Phi
    and the update (for stage-by-stage comparisons)."""
    perm = np.asarray(ordering.perm, dtype=np.int64)
    Ap = permute_csr(A, perm)
    fronts = analyse(Ap, ordering.sep_ptr, ordering.parent)
    updates = {}
    factors = []
    hss_d = {}   # final sample count of each HSS front
    for f in fronts:
        if stop_after is not None and f.id > stop_after:
            break
        idx = f.idx
        if f.s >= opts.min_sep_hss:
            op = FrontOp(Ap, f, fronts, updates)
            orig = perm[idx]

            def rand(c0, nc, orig=orig):
                return gaussian(opts.seed, orig, nc, c0)

            # R_i reuses the random columns of its HSS children (Eq. (Rmerge),
            # Sec. 4.3): it starts with as many as they ended with, at least d0
            d_init = max([opts.d0] + [hss_d[c] for c in f.children if c in hss_d])
            H, F, k, q, Theta, Phi = hs.build_hss_front(
                op, f.s, f.u, opts.leaf_size, rand, opts.rel_tol, d_init, opts.dd, opts.p, opts.d_max,
                opts.abs_tol, opts.power_q, opts.srrqr_f)
            hss_d[f.id] = H.stats["d"]
            data = dict(H=H, ulv=F, k=k, q=q)
            if q >= 0:
                data["ops"] = hs.Front11Ops(H, k, q)
                updates[f.id] = HSSUpdate(H, q, Theta, Phi)
            if record is not None:
                record[f.id] = dict(op=op, rand=rand, H=H, d=H.stats["d"], Theta=Theta, Phi=Phi,
                                    update=updates.get(f.id))
            factors.append(FrontFactor("hss", data))
        else:
            sub = Ap[idx][:, idx].toarray()
            F = np.zeros((f.n, f.n))
            F[:f.s, :] = sub[:f.s, :]
            F[f.s:, :f.s] = sub[f.s:, :f.s]
            for c in f.children:
                dn.extend_add(idx, fronts[c].upd, updates[c].dense(), F)
            res = dn.partial_lu(F, f.s, f.id)
            if f.u:
                updates[f.id] = DenseUpdate(res.pop("U"))
            else:
                res.pop("U")
            factors.append(FrontFactor("dense", res))
        for c in f.children:
            updates.pop(c, None)
    return Factorization(A.n, perm, Ap, fronts, factors, opts)


def apply_inverse(fac, b, trans=False):
    """One application of the multifrontal factors: forward sweep bottom-up,
    backward sweep top-down (Sec. 3.3).  With trans=True the same factors
    solve with A^T.  Dense fronts use P, L11, U11, L21, U12; HSS fronts use
    ULV solves of F11 and the generator products for F21 / F12."""
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    y = b.reshape(b.shape[0], -1)[fac.perm].copy()
    for f, fa in zip(fac.fronts, fac.factors):
        sep = slice(f.sep_lo, f.sep_hi)
        d = fa.data
        if fa.kind == "dense":
            if not trans:
                ys = sla.solve_triangular(d["lu"], y[sep][d["P"]], lower=True, unit_diagonal=True)
                y[sep] = ys
                if f.u:
                    y[f.upd] -= d["L21"] @ ys
            else:
                zs = sla.solve_triangular(d["lu"], y[sep], lower=False, trans=1)
                y[sep] = zs
                if f.u:
                    y[f.upd] -= d["U12"].T @ zs
        else:
            if not trans:
                z = hs.ulv_solve(d["ulv"], y[sep])
                y[sep] = z
                if f.u:
                    y[f.upd] -= d["ops"].f21(z)
            else:
                z = hs.ulv_solve_transpose(d["ulv"], y[sep])
                y[sep] = z
                if f.u:
                    y[f.upd] -= d["ops"].f12t(z)
    for f, fa in zip(reversed(fac.fronts), reversed(fac.factors)):
        sep = slice(f.sep_lo, f.sep_hi)
        d = fa.data
        if fa.kind == "dense":
            if not trans:
                rhs = y[sep] - (d["U12"] @ y[f.upd] if f.u else 0.0)
                y[sep] = sla.solve_triangular(d["lu"], rhs, lower=False)
            else:
                rhs = y[sep] - (d["L21"].T @ y[f.upd] if f.u else 0.0)
                t = sla.solve_triangular(d["lu"], rhs, lower=True, unit_diagonal=True, trans=1)
                out = np.empty_like(t)
                out[d["P"]] = t
                y[sep] = out
        else:
            if f.u:
                if not trans:
                    y[sep] = y[sep] - hs.ulv_solve(d["ulv"], d["ops"].f12(y[f.upd]))
                else:
                    y[sep] = y[sep] - hs.ulv_solve_transpose(d["ulv"], d["ops"].f21t(y[f.upd]))
    x = np.empty_like(y)
    x[fac.perm] = y
    return x[:, 0] if vec else x


def hss_ranks(fac):
    """Per HSS front: (front id, max row rank, max column rank, d, rounds)."""
    out = []
    for f, fa in zip(fac.fronts, fac.factors):
        if fa.kind != "hss":
            continue
        H = fa.data["H"]
        rr = [g.r for g in H.gen if g.UE is not None]
        cc = [g.c for g in H.gen if g.VE is not None]
        out.append((f.id, max(rr, default=0), max(cc, default=0), H.stats["d"], H.stats["rounds"]))
    return out
