"""Seeded synthetic inputs: grid PDE operators, geometric nested dissection,
right-hand sides and coefficient fields.

This module is the only code shared by the oracle and the HIP path.  It holds
none of the solver's arithmetic: it produces the sparse matrix A (CSR, natural
grid ordering), the fill-reducing ordering that both sides consume as an input
(perm, separator tree), and seeded vectors.

Workloads follow the regular-grid PDE benchmarks of the paper (Sec. 6.1):
5-point / 7-point Poisson with homogeneous Dirichlet conditions, an upwind
convection-diffusion operator, and a finite-volume variable-coefficient
diffusion operator.  The ordering is the "geometric nested dissection" the
paper uses for regular grids (Sec. 6.1), made concrete as:

* cut the box along its longest axis (ties to the lower axis index), with the
  separator plane at ``lo + (ext - 1) // 2``;
* stop when every extent is at most ``leaf_side``;
* number fronts in postorder (left subtree, right subtree, separator);
* inside a separator (or a leaf box) order points by recursive coordinate
  bisection (longer side first, first part of size ``ceil(len / 2)``), so a
  run of consecutive indices is a compact patch of the face.  These patches
  play the role of the separator partitions of Sec. 4.2.

For the algebraic front end, :func:`knn_mesh` gives an operator on a random
unstructured point set (no grid, no geometric ordering) and
:func:`permute_rows` scrambles its rows so that static pivoting is needed.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

__all__ = [
    "CSR", "Ordering", "poisson2d", "poisson3d", "convdiff2d", "fv_diffusion3d",
    "smoothed_log_kappa", "geometric_nd", "workload", "WORKLOADS",
]


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int64, n+1
    colind: np.ndarray  # int32, nnz (sorted within a row)
    val: np.ndarray     # float64, nnz

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def matvec(self, x):
        return self.to_scipy() @ x


@dataclass
class Ordering:
    perm: np.ndarray      # int32, perm[new] = old
    sep_ptr: np.ndarray   # int32, nfront+1; front f owns new indices [sep_ptr[f], sep_ptr[f+1])
    parent: np.ndarray    # int32, nfront; -1 for the root; fronts are in postorder
    boxes: list           # per front: (lo, hi) of the subtree box (geometry, informative)
    dims: tuple

    @property
    def nfront(self):
        return len(self.parent)


def _coo_to_csr(n, rows, cols, vals):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


def _grid_index(dims):
    return np.arange(int(np.prod(dims))).reshape(tuple(reversed(dims)))  # [z][y][x]


def _stencil(dims, centre, coeff):
    """Assemble a nearest-neighbour operator on a grid with Dirichlet boundary.

    ``centre`` is an array over grid points (natural ordering x fastest);
    ``coeff(axis, sign)`` returns the off-diagonal value array over grid points
    for the neighbour at +/-1 along ``axis`` (entries whose neighbour falls
    outside the grid are dropped: homogeneous Dirichlet)."""
    dims = tuple(dims)
    n = int(np.prod(dims))
    idx = np.arange(n)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem = rem // d
    stride = np.cumprod((1,) + dims[:-1])
    rows = [idx]
    cols = [idx]
    vals = [np.asarray(centre, dtype=np.float64) * np.ones(n)]
    for ax, d in enumerate(dims):
        for sign in (-1, 1):
            ok = (coords[ax] + sign >= 0) & (coords[ax] + sign < d)
            c = np.asarray(coeff(ax, sign), dtype=np.float64) * np.ones(n)
            rows.append(idx[ok])
            cols.append(idx[ok] + sign * stride[ax])
            vals.append(c[ok])
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def poisson2d(nx, ny=None):
    """5-point Laplacian (4, -1), homogeneous Dirichlet (Sec. 6.1, P2D)."""
    ny = nx if ny is None else ny
    return _stencil((nx, ny), 4.0, lambda ax, s: -1.0)


def poisson3d(nx, ny=None, nz=None):
    """7-point Laplacian (6, -1), homogeneous Dirichlet (Sec. 6.1, P3D)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _stencil((nx, ny, nz), 6.0, lambda ax, s: -1.0)


def convdiff2d(n, wx, wy):
    """-Lap(u) + w.grad(u) with constant w, 5-point first-order upwind, scaled
    by h^2 (h = 1/(n+1)).  Centre 4 + h(|wx|+|wy|); the upwind neighbour gets
    -1 - h|w_axis|, the downwind neighbour -1.  The paper's C2D uses the same
    upwind scheme (Sec. 6.1); the constant field follows the batched workload."""
    h = 1.0 / (n + 1)
    w = (wx, wy)

    def coeff(ax, sign):
        upwind = (sign < 0) if w[ax] >= 0 else (sign > 0)
        return -1.0 - h * abs(w[ax]) if upwind else -1.0

    return _stencil((n, n), 4.0 + h * (abs(wx) + abs(wy)), coeff)


def _velocity(dims, coords):
    """The velocity fields of the paper's convection-diffusion problems
    (Sec. 6.1): in 2D v = (x(1-x)(2y-1), y(1-y)(2x-1)); in 3D
    v = (2x(1-x)(2y-1)z, -y(1-y)(2x-1), -(2x-1)(2y-1)z(1-z))."""
    if len(dims) == 2:
        x, y = coords
        return [x * (1 - x) * (2 * y - 1), y * (1 - y) * (2 * x - 1)]
    x, y, z = coords
    return [2 * x * (1 - x) * (2 * y - 1) * z, -y * (1 - y) * (2 * x - 1), -(2 * x - 1) * (2 * y - 1) * z * (1 - z)]


def convdiff_paper(n, ndim=2, nu=1e-4):
    """The paper's C2D / C3D problems (Sec. 6.1): -nu Lap(u) + v.grad(u) = f on
    the unit square / cube with homogeneous Dirichlet boundary, n interior
    points per side (h = 1/(n+1), point i at (i+1) h), first-order upwind
    differences for the convection and the (2 ndim + 1)-point Laplacian,
    scaled by h^2: centre 2 ndim nu + h sum_a |v_a|, the upwind neighbour
    along axis a -nu - h |v_a|, the downwind one -nu.  nu = 1e-4 as in the
    paper, so convection dominates (cell Peclet numbers up to about 25 at
    n = 100)."""
    dims = (n,) * ndim
    h = 1.0 / (n + 1)
    N = n ** ndim
    idx = np.arange(N)
    coords = []
    rem = idx.copy()
    for _ in dims:
        coords.append((rem % n + 1) * h)
        rem = rem // n
    v = _velocity(dims, coords)

    def coeff(ax, sign):
        up = (v[ax] >= 0) if sign < 0 else (v[ax] < 0)
        return np.where(up, -nu - h * np.abs(v[ax]), -nu)

    return _stencil(dims, 2 * ndim * nu + h * sum(np.abs(va) for va in v), coeff)


@dataclass
class ZCSR:
    """A complex sparse matrix: CSR pattern as in CSR, val complex128."""
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    val: np.ndarray

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))


def helmholtz(n, ndim=2, freq=10.0, ppw=15.0, npml=8, vmin=1500.0, vmax=2500.0):
    """The paper's H2D / H3D problems (Sec. 6.1): (-Lap - omega^2 / v(x)^2) u
    = s on an n^ndim grid, omega = 2 pi freq, h = vmin / (freq ppw) (ppw
    points per wavelength at the slowest velocity), npml layers of
    perfectly matched layer on every side, homogeneous Dirichlet beyond.

    Stretched coordinates s_a = 1 + i sigma_a / omega, sigma_a = sigma0
    (xi / L)^2 at depth xi into a layer of width L = npml h, sigma0 =
    3 vmax ln(10^6) / (2 L); the conservative form -div(D grad u) -
    (omega / v)^2 S u with S = prod_a s_a and D_aa = S / s_a^2 gives a
    complex symmetric matrix.  Stencil: 9 points in 2D, 27 in 3D.  The
    Laplacian is w_1 L_faces + w_2 L_edges (+ w_3 L_corners in 3D), each L_c
    the consistent second difference over the neighbours of its class
    (sum over offsets d of (u(x + h d) - u(x)) divided by h^2 |class| times
    the d d^T trace factor), with the neighbour pair's coefficient
    d^T D d / d^T d taken at the pair's midpoint; the mass term spreads
    (omega / v)^2 S over the same neighbours with weights m_c (centre m_0).
    Velocity v = vmin + (vmax - vmin) times the depth fraction, plus a
    smooth Gaussian anomaly of 10% at the centre."""
    dims = (n,) * ndim
    N = n ** ndim
    omega = 2.0 * np.pi * freq
    h = vmin / (freq * ppw)
    L = npml * h
    sigma0 = 3.0 * vmax * np.log(1e6) / (2.0 * L) if npml > 0 else 0.0
    idx = np.arange(N)
    coords = []
    rem = idx.copy()
    for _ in dims:
        coords.append(rem % n)
        rem = rem // n
    stride = np.array([n ** a for a in range(ndim)])

    def stretch(xa):
        # xa: grid coordinate (may be half-integer); depth into the layers
        if npml == 0:
            return np.ones(np.shape(xa), dtype=np.complex128)
        lo = (npml - 1) - xa
        hi = xa - (n - npml)
        xi = np.maximum(np.maximum(lo, hi), 0.0) * h
        sig = sigma0 * (xi / L) ** 2
        return 1.0 + 1j * sig / omega

    def fields(xs):
        s = [stretch(xa) for xa in xs]
        S = np.prod(s, axis=0)
        D = [S / sa ** 2 for sa in s]
        depth = xs[-1] / max(n - 1, 1)
        r2 = sum(((xa / max(n - 1, 1)) - 0.5) ** 2 for xa in xs)
        v = vmin + (vmax - vmin) * depth + 0.1 * vmin * np.exp(-r2 / 0.02)
        return D, S * (omega / v) ** 2

    offs = [np.array(d) for d in np.ndindex(*(3,) * ndim)]
    offs = [d - 1 for d in offs if np.any(d != 1)]
    if ndim == 2:
        lap_w = {1: 0.6, 2: 0.4}
        mass_w = {0: 0.6, 1: 0.08, 2: 0.02}
    else:
        lap_w = {1: 0.6, 2: 0.3, 3: 0.1}
        mass_w = {0: 0.5, 1: 0.05, 2: 0.01, 3: 0.0025}
    # trace factor: sum over a class's offsets of d d^T = t_c I
    tr = {c: sum(int(np.sum(d != 0) == c) * (np.abs(d) > 0) for d in offs)[0] for c in lap_w}
    rows, cols, vals = [], [], []
    centre = np.zeros(N, dtype=np.complex128)
    D0, K0 = fields([c.astype(np.float64) for c in coords])
    centre -= mass_w[0] * K0
    for d in offs:
        c = int(np.sum(d != 0))
        ok = np.ones(N, dtype=bool)
        for a in range(ndim):
            ok &= (coords[a] + d[a] >= 0) & (coords[a] + d[a] < n)
        mid = [coords[a][ok] + 0.5 * d[a] for a in range(ndim)]
        Dm, Km = fields(mid)
        ddd = sum(Dm[a] * d[a] * d[a] for a in range(ndim)) / float(d @ d)
        lap = -lap_w[c] / (tr[c] * h * h) * 2.0 * ddd
        mass = -mass_w[c] * Km
        off = lap + mass
        src = idx[ok]
        rows.append(src)
        cols.append(src + int(d @ stride))
        vals.append(off)
        np.add.at(centre, src, -lap)
    rows.append(idx)
    cols.append(idx)
    vals.append(centre)
    r = np.concatenate(rows)
    cc = np.concatenate(cols)
    vv = np.concatenate(vals)
    order = np.lexsort((cc, r))
    r, cc, vv = r[order], cc[order], vv[order]
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    return ZCSR(N, np.cumsum(rowptr), cc.astype(np.int32), vv.astype(np.complex128))


def smoothed_log_kappa(n, seed=3, sigma=0.5):
    """log(kappa) iid N(0, sigma^2) from ``default_rng(seed)``, then a 3x3x3 box
    mean over the in-domain neighbours.  Returns (kappa, rng) so that the caller
    can keep drawing from the same stream (b, then x*)."""
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, sigma, n ** 3).reshape(n, n, n)  # [z][y][x]
    s = np.zeros_like(g)
    c = np.zeros_like(g)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                src = [slice(max(0, -d), n - max(0, d)) for d in (dz, dy, dx)]
                dst = [slice(max(0, d), n - max(0, -d)) for d in (dz, dy, dx)]
                s[tuple(dst)] += g[tuple(src)]
                c[tuple(dst)] += 1.0
    return np.exp(s / c).reshape(-1), rng


def fv_diffusion3d(n, kappa):
    """Cell-centred finite-volume -div(kappa grad u) on an n^3 grid with unit
    spacing: face transmissibility 2 k_c k_c' / (k_c + k_c'); a Dirichlet
    boundary face contributes 2 k_c to the diagonal."""
    dims = (n, n, n)
    N = n ** 3
    kappa = np.asarray(kappa, dtype=np.float64)
    idx = np.arange(N)
    coords = [idx % n, (idx // n) % n, idx // (n * n)]
    stride = (1, n, n * n)
    diag = np.zeros(N)
    rows, cols, vals = [], [], []
    for ax in range(3):
        for sign in (-1, 1):
            ok = (coords[ax] + sign >= 0) & (coords[ax] + sign < n)
            nb = idx[ok] + sign * stride[ax]
            kc, kn = kappa[idx[ok]], kappa[nb]
            t = 2.0 * kc * kn / (kc + kn)
            rows.append(idx[ok]); cols.append(nb); vals.append(-t)
            np.add.at(diag, idx[ok], t)
            np.add.at(diag, idx[~ok], 2.0 * kappa[idx[~ok]])
    rows.append(idx); cols.append(idx); vals.append(diag)
    return _coo_to_csr(N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def fv_diffusion3d_values(n, kappa):
    """The CSR values of :func:`fv_diffusion3d` (same order) as a function of
    ``kappa`` written with torch operations, so that a loss computed from the
    solution can be differentiated with respect to the coefficients by
    automatic differentiation through the assembly (the chain rule from
    dL/dval to dL/dkappa)."""
    import torch
    N = n ** 3
    idx = np.arange(N)
    coords = [idx % n, (idx // n) % n, idx // (n * n)]
    stride = (1, n, n * n)
    dev = kappa.device
    diag = torch.zeros(N, dtype=kappa.dtype, device=dev)
    rows, cols, vals = [], [], []
    for ax in range(3):
        for sign in (-1, 1):
            ok = (coords[ax] + sign >= 0) & (coords[ax] + sign < n)
            a = idx[ok]
            nb = a + sign * stride[ax]
            ta = torch.as_tensor(a, device=dev)
            kc, kn = kappa[ta], kappa[torch.as_tensor(nb, device=dev)]
            t = 2.0 * kc * kn / (kc + kn)
            rows.append(a); cols.append(nb); vals.append(-t)
            diag = diag.index_add(0, ta, t)
            bd = torch.as_tensor(idx[~ok], device=dev)
            diag = diag.index_add(0, bd, 2.0 * kappa[bd])
    rows.append(idx); cols.append(idx); vals.append(diag)
    order = np.lexsort((np.concatenate(cols), np.concatenate(rows)))
    return torch.cat(vals)[torch.as_tensor(order, device=dev)]


# ---------------------------------------------------------------------------
# geometric nested dissection
# ---------------------------------------------------------------------------

@lru_cache(maxsize=None)
def _rcb_shape(shape):
    """Relative coordinates of a box of ``shape`` in recursive coordinate
    bisection order: split the longest side (ties to the lower axis) with the
    first part holding ceil(len/2) points, recurse down to single points."""
    size = int(np.prod(shape))
    if size == 1:
        return np.zeros((1, len(shape)), dtype=np.int64)
    ax = int(np.argmax(shape))
    first = (shape[ax] + 1) // 2
    s1 = list(shape); s1[ax] = first
    s2 = list(shape); s2[ax] = shape[ax] - first
    a = _rcb_shape(tuple(s1))
    b = _rcb_shape(tuple(s2)).copy()
    b[:, ax] += first
    return np.concatenate([a, b], axis=0)


def _box_points(lo, hi, dims):
    shape = tuple(int(h - l) for l, h in zip(lo, hi))
    rel = _rcb_shape(shape)
    absc = rel + np.asarray(lo, dtype=np.int64)
    stride = np.cumprod((1,) + tuple(dims[:-1]))
    return (absc * stride).sum(axis=1)


def geometric_nd(dims, leaf_side):
    """Nested dissection of a regular grid (see module docstring).  Returns an
    :class:`Ordering`; fronts are numbered in postorder."""
    dims = tuple(int(d) for d in dims)
    fronts_pts = []
    parent = []
    boxes = []

    def rec(lo, hi):
        ext = [h - l for l, h in zip(lo, hi)]
        if min(ext) <= 0:
            return -1
        if max(ext) <= leaf_side:
            fid = len(fronts_pts)
            fronts_pts.append(_box_points(lo, hi, dims))
            parent.append(-1)
            boxes.append((tuple(lo), tuple(hi)))
            return fid
        ax = int(np.argmax(ext))
        cut = lo[ax] + (ext[ax] - 1) // 2
        hl = list(hi); hl[ax] = cut
        lr = list(lo); lr[ax] = cut + 1
        a = rec(list(lo), hl)
        b = rec(lr, list(hi))
        slo = list(lo); slo[ax] = cut
        shi = list(hi); shi[ax] = cut + 1
        fid = len(fronts_pts)
        fronts_pts.append(_box_points(slo, shi, dims))
        parent.append(-1)
        boxes.append((tuple(lo), tuple(hi)))
        for c in (a, b):
            if c >= 0:
                parent[c] = fid
        return fid

    import sys
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 10000))
    try:
        rec([0] * len(dims), list(dims))
    finally:
        sys.setrecursionlimit(old)
    sizes = np.array([len(p) for p in fronts_pts], dtype=np.int64)
    sep_ptr = np.zeros(len(sizes) + 1, dtype=np.int32)
    sep_ptr[1:] = np.cumsum(sizes)
    perm = np.concatenate(fronts_pts).astype(np.int32)
    return Ordering(perm, sep_ptr, np.asarray(parent, dtype=np.int32), boxes, dims)


def halo_size(box, dims):
    """Number of grid points just outside ``box`` across its faces (no edges
    or corners) that lie inside the grid: the update-set size of the front
    whose subtree covers ``box`` for a 5-/7-point stencil."""
    lo, hi = box
    ext = [h - l for l, h in zip(lo, hi)]
    tot = 0
    for ax in range(len(dims)):
        area = int(np.prod([e for b, e in enumerate(ext) if b != ax]))
        if lo[ax] > 0:
            tot += area
        if hi[ax] < dims[ax]:
            tot += area
    return tot


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (kind, grid side, nd leaf side, solver options)
    "poisson2d_100": dict(kind="poisson2d", n=100, leaf_side=8,
                          opts=dict(min_sep_hss=64, leaf_size=16, rel_tol=1e-4, d0=32, dd=16,
                                    outer="gmres")),
    "poisson3d_64": dict(kind="poisson3d", n=64, leaf_side=4,
                         opts=dict(min_sep_hss=512, leaf_size=64, rel_tol=1e-6, d0=128, dd=128,
                                   outer="ir")),
}


def workload(kind, n, leaf_side, rhs_seed=1, **_):
    """Matrix, ordering and right-hand side of a named grid workload.  The
    right-hand side is iid N(0,1) from ``default_rng(rhs_seed)``."""
    if kind == "poisson2d":
        A = poisson2d(n)
        order = geometric_nd((n, n), leaf_side)
    elif kind == "poisson3d":
        A = poisson3d(n)
        order = geometric_nd((n, n, n), leaf_side)
    else:
        raise ValueError(kind)
    b = np.random.default_rng(rhs_seed).standard_normal(A.n)
    return A, order, b


def knn_mesh(npts, k=6, seed=0, wind=(0.6, -0.3), shift=1e-2):
    """An unstructured-mesh operator for the algebraic front end: npts
    points uniform in the unit square (``default_rng(seed)``), each joined
    to its k nearest neighbours (edges symmetrized); a_ij = -1 - w.(x_j - x_i)
    / |x_j - x_i| * 0.5 on every edge (a graph Laplacian with a skew
    convection term along ``wind``), a_ii = degree + shift.  Diagonally
    dominant, nonsymmetric, no geometric grid.  Returns (CSR, points)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (npts, 2))
    _, nb = cKDTree(pts).query(pts, k + 1)
    rows = np.repeat(np.arange(npts), k)
    cols = nb[:, 1:].ravel()
    e = np.unique(np.concatenate([np.stack([rows, cols], 1), np.stack([cols, rows], 1)]), axis=0)
    i, j = e[:, 0], e[:, 1]
    d = pts[j] - pts[i]
    skew = 0.5 * (d @ np.asarray(wind, dtype=np.float64)) / np.linalg.norm(d, axis=1)
    off = -1.0 - skew
    deg = np.bincount(i, minlength=npts).astype(np.float64)
    rr = np.concatenate([i, np.arange(npts)])
    cc = np.concatenate([j, np.arange(npts)])
    vv = np.concatenate([off, deg + shift])
    return _coo_to_csr(npts, rr, cc, vv), pts


def permute_rows(A, seed):
    """P A for a random row permutation P (``default_rng(seed)``): the
    diagonal of the result is mostly zero."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(A.n)
    S = A.to_scipy()[p].tocoo()
    return _coo_to_csr(A.n, S.row, S.col, S.data)


def convdiff_batch(count=256, seed=2, side_lo=48, side_hi=160, wmax=20.0, leaf_side=8):
    """Independent 2D convection-diffusion systems of uneven sizes: with
    ``rng = default_rng(seed)``, sides ``n_j = rng.integers(side_lo,
    side_hi + 1, count)``, speeds ``|w_j| = rng.uniform(0, wmax, count)``,
    angles ``theta_j = rng.uniform(0, 2 pi, count)``, then right-hand sides
    ``b_j = rng.standard_normal(n_j^2)`` in order of j.  Each system is the
    upwind operator of :func:`convdiff2d` with w = |w|(cos theta, sin theta),
    ordered by :func:`geometric_nd` with ``leaf_side``.  Returns a list of
    (A, ordering, b)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, count)
    speed = rng.uniform(0.0, wmax, count)
    theta = rng.uniform(0.0, 2.0 * np.pi, count)
    out = []
    for j in range(count):
        n = int(sides[j])
        A = convdiff2d(n, float(speed[j] * np.cos(theta[j])), float(speed[j] * np.sin(theta[j])))
        out.append([A, geometric_nd((n, n), leaf_side), None])
    for j in range(count):
        out[j][2] = rng.standard_normal(int(sides[j]) ** 2)
    return [tuple(t) for t in out]
