"""Symbolic analysis (oracle side): fronts, update index sets, HSS trees.

Fronts follow the amalgamated elimination tree of a nested-dissection
ordering: one front per separator (Sec. 3.1).  Front i has index set
I_i = {I_sep_i, I_upd_i} (Eq. frontal_1); I_upd_i is the standard symbolic
rule: the union of the children's update sets and of the indices j after the
separator with A(I_sep, j) != 0 or A(j, I_sep) != 0, minus I_sep.

Per HSS front, the HSS tree (Sec. 2.1) is a postordered binary tree over the
front's local indices.  If the front has an update part, the root's children
are k (the separator block F11) and q (the update block F22); each part is
split recursively by halving its count (left part ceil(n/2)) until a node
holds at most ``leaf_size`` indices.  A front without update part uses the
separator tree alone.  Nodes own contiguous ranges (Sec. 2.1).
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Front:
    id: int
    sep_lo: int
    sep_hi: int
    upd: np.ndarray          # sorted new indices (int64)
    children: list
    parent: int

    @property
    def s(self):
        return self.sep_hi - self.sep_lo

    @property
    def u(self):
        return len(self.upd)

    @property
    def n(self):
        return self.s + self.u

    @property
    def idx(self):
        return np.concatenate([np.arange(self.sep_lo, self.sep_hi), self.upd])


def permute_csr(A, perm):
    """P A P^T as a scipy CSR with sorted indices, where perm[new] = old."""
    S = A.to_scipy()
    B = S[perm][:, perm].tocsr()
    B.sort_indices()
    return B


def analyse(Ap, sep_ptr, parent):
    """Fronts (postorder) with update sets, from the permuted matrix Ap."""
    nf = len(parent)
    children = [[] for _ in range(nf)]
    for f in range(nf):
        if parent[f] >= 0:
            children[parent[f]].append(f)
    sym = (Ap + Ap.T).tocsr()
    sym.sort_indices()
    fronts = []
    for f in range(nf):
        lo, hi = int(sep_ptr[f]), int(sep_ptr[f + 1])
        cols = sym.indices[sym.indptr[lo]:sym.indptr[hi]]
        parts = [cols[cols >= hi].astype(np.int64)]
        for c in children[f]:
            up = fronts[c].upd
            parts.append(up[up >= hi])
        upd = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
        fronts.append(Front(f, lo, hi, upd, children[f], int(parent[f])))
    return fronts


@dataclass
class HNode:
    lo: int
    hi: int
    children: list = field(default_factory=list)   # node ids (postorder numbering)
    parent: int = -1

    @property
    def m(self):
        return self.hi - self.lo

    @property
    def leaf(self):
        return not self.children


def _split(nodes, lo, hi, leaf_size):
    if hi - lo <= leaf_size:
        nodes.append(HNode(lo, hi))
        return len(nodes) - 1
    mid = lo + (hi - lo + 1) // 2
    a = _split(nodes, lo, mid, leaf_size)
    b = _split(nodes, mid, hi, leaf_size)
    nodes.append(HNode(lo, hi, [a, b]))
    nodes[a].parent = nodes[b].parent = len(nodes) - 1
    return len(nodes) - 1


def hss_tree(s, u, leaf_size):
    """Postordered HSS tree of a front with separator size s and update size
    u.  Returns (nodes, k, q): k/q are the F11 / F22 subtree roots (q = -1 when
    u == 0, in which case k is the root)."""
    nodes = []
    k = _split(nodes, 0, s, leaf_size)
    if u == 0:
        return nodes, k, -1
    q = _split(nodes, s, s + u, leaf_size)
    nodes.append(HNode(0, s + u, [k, q]))
    nodes[k].parent = nodes[q].parent = len(nodes) - 1
    return nodes, k, q
