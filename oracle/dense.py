"""Dense-front kernels of the multifrontal method (oracle side, FP64).

Sec. 3.2: a frontal matrix F = [F11 F12; F21 F22] is assembled from the
original entries and the children's update matrices by extend-add
(Eq. extend-add), then F11 is factored with partial pivoting restricted to
F11 (no delayed pivoting, Sec. 3.2) and the update matrix
U = F22 - F21 F11^{-1} F12 is formed.
"""
import numpy as np
import scipy.linalg as sla


class SingularFront(ArithmeticError):
    def __init__(self, front):
        super().__init__(f"zero pivot in front {front}")
        self.front = front


def extend_add(parent_idx, child_idx, Uc, F):
    """F += extend(Uc): Uc is indexed by the (sorted) global indices
    ``child_idx``, F by ``parent_idx``; child_idx must be a subset of
    parent_idx.  Plain indexed summation (Eq. extend-add)."""
    pos = np.searchsorted(parent_idx, child_idx)
    assert np.all(parent_idx[pos] == child_idx)
    F[np.ix_(pos, pos)] += Uc


def partial_lu(F, s, front_id=-1):
    """Partial factorization of an assembled front F (n x n) with separator
    size s.  Returns dict with the getrf factors of F11 (lu, piv), L21 =
    F21 U11^{-1}, U12 = L11^{-1} P F12 and the update matrix U."""
    F11 = F[:s, :s]
    lu, piv = sla.lu_factor(F11, check_finite=True)
    if s and np.any(np.diag(lu) == 0.0):
        raise SingularFront(front_id)
    P = np.arange(s)
    for i, pv in enumerate(piv):
        P[[i, pv]] = P[[pv, i]]
    L11 = np.tril(lu, -1) + np.eye(s)
    U11 = np.triu(lu)
    U12 = sla.solve_triangular(L11, F[:s, s:][P], lower=True, unit_diagonal=True)
    L21 = sla.solve_triangular(U11, F[s:, :s].T, lower=False, trans=1).T
    Uupd = F[s:, s:] - L21 @ U12
    return dict(lu=lu, piv=piv, P=P, L21=L21, U12=U12, U=Uupd)
