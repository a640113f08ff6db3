"""Algorithmic work of a factorization and of one preconditioner
application, counted from the oracle's own results (TEST INFRASTRUCTURE:
these counts price the GPU's measured times against the machine's peaks).

The counts are the operations the method itself has to perform, per stage,
not those of any particular implementation:

- dense front (s, u): 2/3 s^3 + 2 s^2 u + 2 s u^2 flops (partial LU with the
  Schur update, Sec. 3.2); HBM traffic: the front read and written once,
  24 (s + u)^2 bytes;
- extend-add of a child's update matrix into a dense parent (Eq.
  extend-add): u^2 flops, 24 u^2 bytes (read child, read and write parent);
- assembly of a dense front: 8 (s + u)^2 bytes of zero fill plus 24 bytes per
  original entry (value, index, destination);
- sampling S^r = F R, S^c = F^T R by skinny extend-add (Eq. FtimesR, Sec. 4.3)
  for w new columns: 4 nnz(A_i) w for the original entries; 4 u^2 w for a
  dense child; for an HSS child, the HSS matvec of its F22 block in both
  directions plus Theta^* (Phi X) (Sec. 4.4); HBM traffic: each dense child
  matrix read once per pass (8 u^2), R read and both samples written
  (24 n w);
- ID of a d x m sample block truncated at rank k (Sec. 2.2, Sec. 5.3):
  Householder QR 4 d m k - 2 k^2 (d + m) + 4/3 k^3, then the triangular solve
  for E, k^2 (m - k); traffic: the block read once, 8 d m bytes;
- sample updates of Alg. 1: leaf 4 m^2 w (D R, D^T R), non-leaf
  4 (r1 c2 + r2 c1) w (B R), and the random-matrix reductions
  2 (m - k) k w per side;
- ULV of every node of the F11 subtree (Sec. 2.3), with p = m - r:
  2 p r m (Omega D), 2 p^2 (m - p/3) (the LQ of the top rows) and
  4 p m (r + c) (Q applied to the rest); 2/3 m_k^3 for the LU at the top
  node; the low-rank Schur factors Theta^*, Phi (Sec. 4.4);
- one application of M^{-1}: every stored factor word read once (HBM bound,
  Sec. 6.2 reports the solve at the memory bandwidth); SpMV 12 bytes per
  nonzero plus 24 bytes per unknown.
"""
import numpy as np

from . import hss as hs


STAGES = ("dense_lu", "extend_add", "assembly", "sampling", "id", "sample_update", "ulv", "schur")


def _tree_shapes(H):
    """Per node: (leaf, m, r, c, children) with the final generators."""
    out = {}
    for t, nd in enumerate(H.nodes):
        g = H.gen[t]
        out[t] = (nd.leaf, nd.m, g.r if g.UE is not None else 0, g.c if g.VE is not None else 0,
                  tuple(nd.children))
    return out


def _hss_matvec_flops(H, rt, w):
    """Flops of Y = F X and Y = F^T X together on the subtree of rt for w
    columns: up-sweep, sibling products, down-sweep, leaf diagonal blocks."""
    sh = _tree_shapes(H)
    fl = 0.0
    for t in hs._subtree(H.nodes, rt):
        leaf, m, r, c, ch = sh[t]
        if leaf:
            fl += 2.0 * m * m * w
        if t != rt:
            mm = m if leaf else (sh[ch[0]][2] + sh[ch[1]][2])
            mc = m if leaf else (sh[ch[0]][3] + sh[ch[1]][3])
            fl += 2.0 * mc * c * w + 2.0 * mm * r * w    # V^T x up, U y down
        if not leaf:
            a, b = ch
            fl += 2.0 * (sh[a][2] * sh[b][3] + sh[b][2] * sh[a][3]) * w
    return 2.0 * fl   # F and F^T


def id_flops(d, m, k):
    """Householder QR of a d x m block truncated at k columns, plus the
    triangular solve for E (Sec. 2.2)."""
    return 4.0 * d * m * k - 2.0 * k * k * (d + m) + 4.0 / 3.0 * k ** 3 + k * k * (m - k)


class Tally:
    def __init__(self):
        self.flops = {s: 0.0 for s in STAGES}
        self.bytes = {s: 0.0 for s in STAGES}

    def add(self, stage, flops, nbytes):
        self.flops[stage] += float(flops)
        self.bytes[stage] += float(nbytes)

    def as_dict(self):
        return {s: {"flops": self.flops[s], "bytes": self.bytes[s]} for s in STAGES}


def factorization_work(fac):
    """Per-stage algorithmic flops and HBM bytes of the numeric factorization
    ``fac`` (an ``oracle.mf.Factorization``)."""
    T = Tally()
    fronts = fac.fronts
    kinds = {f.id: fa.kind for f, fa in zip(fronts, fac.factors)}
    hss_of = {f.id: fa.data for f, fa in zip(fronts, fac.factors) if fa.kind == "hss"}
    Ap = fac.Ap.tocsr()
    for f, fa in zip(fronts, fac.factors):
        s, u, n = f.s, f.u, f.n
        idx = f.idx
        sub = Ap[idx][:, idx].tocoo()
        nnz_i = int(np.sum((sub.row < s) | (sub.col < s)))
        if fa.kind == "dense":
            T.add("dense_lu", 2.0 / 3.0 * s ** 3 + 2.0 * s * s * u + 2.0 * s * u * u, 24.0 * n * n)
            T.add("assembly", 0.0, 8.0 * n * n + 24.0 * nnz_i)
            for c in f.children:
                uc = fronts[c].u
                T.add("extend_add", uc * uc, 24.0 * uc * uc)
            continue
        d = fa.data
        H = d["H"]
        log = H.stats["log"]
        sh = _tree_shapes(H)
        # sampling passes (initial d, then dd per growth round)
        for w in log["sampled"]:
            fl = 4.0 * nnz_i * w
            by = 24.0 * n * w + 12.0 * nnz_i
            for c in f.children:
                uc = fronts[c].u
                if kinds[c] == "dense":
                    fl += 4.0 * uc * uc * w
                    by += 8.0 * uc * uc
                else:
                    cd = hss_of[c]
                    Hc, q = cd["H"], cd["q"]
                    mk = cd["ulv"].lu[0].shape[0]
                    fl += _hss_matvec_flops(Hc, q, w) + 2.0 * (2.0 * uc * mk * w) * 2.0
            T.add("sampling", fl, by)
        # IDs, every attempt (growth rounds redo failed nodes)
        for (t, dd, mr, kr, mc, kc) in log["ids"]:
            for m, k in ((mr, kr), (mc, kc)):
                T.add("id", id_flops(dd, m, k), 8.0 * dd * m)
            leaf, mm, r, c, ch = sh[t]
            if leaf:
                T.add("sample_update", 4.0 * mm * mm * dd, 8.0 * (mm * mm + 3 * mm * dd))
            else:
                a, b = ch
                T.add("sample_update", 4.0 * (sh[a][2] * sh[b][3] + sh[b][2] * sh[a][3]) * dd,
                      8.0 * 3 * (mr + mc) * dd)
        # random-matrix reductions of successful nodes (and their refresh on
        # new columns, with the leaf / B sample updates of those columns)
        succ = {}
        for (t, w) in log["node_cols"]:
            leaf, mm, r, c, ch = sh[t]
            mr = mm if leaf else sh[ch[0]][2] + sh[ch[1]][2]
            mc = mm if leaf else sh[ch[0]][3] + sh[ch[1]][3]
            T.add("sample_update", 2.0 * (mr - r) * r * w + 2.0 * (mc - c) * c * w, 8.0 * (mr + mc) * w)
            if t in succ:   # a refresh: the node samples of the new columns too
                if leaf:
                    T.add("sample_update", 4.0 * mm * mm * w, 8.0 * 3 * mm * w)
                else:
                    a, b = ch
                    T.add("sample_update", 4.0 * (sh[a][2] * sh[b][3] + sh[b][2] * sh[a][3]) * w,
                          8.0 * 3 * (mr + mc) * w)
            succ[t] = True
        # ULV of the F11 subtree and the top LU
        ulv = d["ulv"]
        for t, un in ulv.nodes.items():
            m, r = un.m, un.r
            c = sh[t][3]
            p = m - r
            T.add("ulv", 2.0 * p * r * m + 2.0 * p * p * (m - p / 3.0) + 4.0 * p * m * (r + c),
                  8.0 * (2 * m * m + m * c))
        mk = ulv.lu[0].shape[0]
        T.add("ulv", 2.0 / 3.0 * mk ** 3, 8.0 * mk * mk * 2)
        if d["q"] >= 0:
            k, q = d["k"], d["q"]
            rq, cq = sh[q][2], sh[q][3]
            rk, ck = sh[k][2], sh[k][3]
            th = 2.0 * u * rq * ck + 2.0 * u * ck * mk + u * mk * mk
            ph = 2.0 * mk * rk * cq + 2.0 * mk * cq * u + mk * mk * u
            T.add("schur", th + ph, 8.0 * 2 * u * mk)
    return T.as_dict()


def _words(a):
    return 0 if a is None else int(np.asarray(a).size)


def apply_bytes(fac):
    """HBM bytes of one application of M^{-1}: every stored factor word read
    once (dense fronts: LU of F11, L21, U12; HSS fronts: the ULV factors, the
    generators and the top LU), plus the right-hand side read and written
    once per front it touches."""
    words = 0
    vec = 0
    for f, fa in zip(fac.fronts, fac.factors):
        d = fa.data
        vec += 2 * (f.s + f.u)
        if fa.kind == "dense":
            words += _words(d["lu"]) + _words(d["L21"]) + _words(d["U12"])
            continue
        H = d["H"]
        for g in H.gen:
            words += _words(g.D) + _words(g.B12) + _words(g.B21) + _words(g.UE) + _words(g.VE)
        for un in d["ulv"].nodes.values():
            words += _words(un.L) // 2 + _words(un.Q) + _words(un.D21) + _words(un.V1) + _words(un.E)
        words += _words(d["ulv"].lu[0])
    return 8.0 * (words + vec)


def spmv_bytes(A):
    return 12.0 * float(A.rowptr[-1]) + 24.0 * float(A.n)
