"""Outer solvers (oracle side, FP64).

The paper uses the (approximate) multifrontal factorization as a
preconditioner for restarted GMRES(30) with modified Gram-Schmidt and a zero
initial guess, and iterative refinement when no HSS is used (Sec. 4.6,
Sec. 6.1).  Reading of the stopping rule: stop on the true relative residual
||b - A x||_2 / ||b||_2 <= tol (the paper tests the preconditioned residual);
GMRES checks it whenever its preconditioned estimate has dropped by tol and
at every restart.
"""
import numpy as np


class NoConvergence(RuntimeError):
    def __init__(self, x, relres, its):
        super().__init__(f"no convergence: relres={relres:.3e} after {its} iterations")
        self.x, self.relres, self.its = x, relres, its


def refine(matvec, prec, b, tol, max_it=50):
    """Iterative refinement: x = M^{-1} b; r = b - A x; x += M^{-1} r."""
    nb = np.linalg.norm(b)
    x = prec(b)
    hist = []
    for it in range(max_it + 1):
        r = b - matvec(x)
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            return x, it, hist
        if it == max_it:
            break
        x = x + prec(r)
    raise NoConvergence(x, hist[-1], max_it)


def gmres(matvec, prec, b, tol, restart=30, max_it=300, x0=None):
    """Left-preconditioned restarted GMRES(m) with modified Gram-Schmidt
    Arnoldi and Givens rotations, x0 = 0 unless given."""
    n = b.shape[0]
    nb = np.linalg.norm(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    its = 0
    hist = []
    while its < max_it:
        r = prec(b - matvec(x))
        beta = np.linalg.norm(r)
        if its == 0:
            beta0 = beta
        V = np.zeros((n, restart + 1))
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        converged = False
        for j in range(restart):
            w = prec(matvec(V[:, j]))
            for i in range(j + 1):
                Hm[i, j] = np.dot(w, V[:, i])
                w = w - Hm[i, j] * V[:, i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0:
                V[:, j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / den
            sn[j] = Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            if abs(g[j + 1]) <= tol * beta0 or its >= max_it or Hm[j, j] == 0:
                y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), g[:j_done])
                xt = x + V[:, :j_done] @ y
                rel = np.linalg.norm(b - matvec(xt)) / nb
                hist.append(rel)
                if rel <= tol:
                    return xt, its, hist
                if its >= max_it:
                    break
        y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), g[:j_done])
        x = x + V[:, :j_done] @ y
        rel = np.linalg.norm(b - matvec(x)) / nb
        hist.append(rel)
        if rel <= tol:
            return x, its, hist
        if converged:
            break
    raise NoConvergence(x, hist[-1] if hist else np.inf, its)


def refine_or_gmres(matvec, prec, b, tol, max_it=50, restart=30):
    """Iterative refinement that hands over to GMRES(restart) when it
    stagnates: once the relative residual has failed to fall below 0.9 times
    the previous one on two consecutive steps, GMRES continues from the
    current iterate with the same preconditioner (a weak preconditioner,
    e.g. an HSS factorization at a large tolerance, need not be a
    contraction, which refinement requires, while GMRES only needs it to
    cluster the spectrum; Sec. 4.6).  Returns (x, iterations, history,
    switched): iterations counts refinement steps plus GMRES iterations."""
    nb = np.linalg.norm(b)
    x = prec(b)
    hist = []
    slow = 0
    for it in range(max_it + 1):
        r = b - matvec(x)
        rel = np.linalg.norm(r) / nb
        if hist and rel > 0.9 * hist[-1]:
            slow += 1
        else:
            slow = 0
        hist.append(rel)
        if rel <= tol:
            return x, it, hist, False
        if slow >= 2 or it == max_it:
            break
        x = x + prec(r)
    if slow < 2:
        raise NoConvergence(x, hist[-1], max_it)
    xg, its, gh = gmres(matvec, prec, b, tol, restart=restart, max_it=max_it, x0=x)
    return xg, it + its, hist + gh, True
