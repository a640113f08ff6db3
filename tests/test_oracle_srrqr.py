"""Pins for the oracle's strong rank-revealing QR (Gu and Eisenstat 1996,
the rank held fixed), the replacement of the column-pivoted QR inside the
ID that Sec. 2.2 and Sec. 7 name (CPU only).

Every check here is computed without the oracle's own formulas for the
interchange criterion: selections are judged by their volumes
sqrt(det(Y_J^T Y_J)) (a Gram determinant per candidate selection, by brute
force), by the singular values of Y (a library SVD), and by the ID's
reconstruction of Y."""
import itertools

import numpy as np
import pytest

from oracle import hss as H


def _logvol(Y, J):
    """log of the volume of the columns J of Y: half the log Gram determinant."""
    G = Y[:, J].T @ Y[:, J]
    sign, ld = np.linalg.slogdet(G)
    assert sign > 0
    return 0.5 * ld


def _kahan(n, c):
    """Kahan's matrix diag(1, s, .., s^(n-1)) (I - c N), N strictly upper
    ones, s^2 + c^2 = 1, with column j scaled by 1 - 1e-10 j so that the
    column-pivoted QR takes the columns in their order (every column of the
    unscaled matrix has norm 1)."""
    s = np.sqrt(1.0 - c * c)
    T = np.eye(n) - c * np.triu(np.ones((n, n)), 1)
    K = np.diag(s ** np.arange(n)) @ T
    return K * (1.0 - 1e-10 * np.arange(n))[None, :]


def _no_volume_gain_above(Y, J, f, rel=1e-9):
    """Brute force: no single interchange of a column of J with one outside
    J multiplies the volume by more than f."""
    m = Y.shape[1]
    rest = [j for j in range(m) if j not in set(J)]
    base = _logvol(Y, J)
    worst = -np.inf
    for a, b in itertools.product(range(len(J)), rest):
        J2 = list(J)
        J2[a] = b
        worst = max(worst, _logvol(Y, J2) - base)
    return worst <= np.log(f) + rel, worst


def test_kahan_matrix_swaps_and_meets_the_bounds():
    """On Kahan's matrix the column-pivoted QR keeps the natural order and
    its interpolation coefficients R11^{-1} R12 grow like (1 + c)^n; with
    k = n - 1 the strong RRQR must interchange columns, after which every
    coefficient is at most f, no single interchange gains volume by more
    than f, and the singular-value bounds of Gu and Eisenstat (Thm. 3.2)
    hold: sigma_i(R11) >= sigma_i(Y) / sqrt(1 + f^2 k (n - k)) and
    ||R22|| <= sigma_{k+1}(Y) sqrt(1 + f^2 k (n - k))."""
    n, c, f = 24, 0.3, 2.0
    K = _kahan(n, c)
    sv = np.linalg.svd(K, compute_uv=False)
    perm0, R0, k = H.cpqr_eps(K, 1e-300)
    assert k == n and np.array_equal(perm0, np.arange(n))
    k = n - 1
    X0 = np.linalg.solve(np.triu(R0[:k, :k]), R0[:k, k:])
    assert np.max(np.abs(X0)) > 10 * f
    perm, W, swaps = H.strong_rrqr(K, perm0, k, f)
    assert swaps >= 1
    J = list(perm[:k])
    X = np.linalg.solve(np.triu(W[:k, :k]), W[:k, k:])
    assert np.max(np.abs(X)) <= f * (1 + 1e-12)
    ok, worst = _no_volume_gain_above(K, J, f)
    assert ok, worst
    bound = np.sqrt(1.0 + f * f * k * (n - k))
    s11 = np.linalg.svd(np.triu(W[:k, :k]), compute_uv=False)
    assert np.all(s11 >= sv[:k] / bound * (1 - 1e-10))
    assert np.linalg.norm(W[k:, k:], 2) <= sv[k] * bound * (1 + 1e-10)
    # the selection of the column-pivoted QR fails the last bound by far
    assert abs(R0[k, k]) > 10 * sv[k] * bound


@pytest.mark.parametrize("seed,d,m,f", [(1, 12, 20, 1.01), (2, 20, 12, 1.01), (3, 16, 16, 1.2), (4, 10, 30, 1.05)])
def test_final_selection_has_no_interchange_gaining_more_than_f(seed, d, m, f):
    """Random matrices with a decaying spectrum and near-duplicate columns
    (where the greedy pivot choice is not volume-optimal): after the
    strong RRQR no single interchange gains volume by more than f, by brute
    force over all k (m - k) interchanges, and every interpolation
    coefficient is at most f."""
    rg = np.random.default_rng(seed)
    r = min(d, m)
    U = np.linalg.qr(rg.standard_normal((d, r)))[0]
    V = np.linalg.qr(rg.standard_normal((m, r)))[0]
    Y = U @ np.diag(0.5 ** np.arange(r)) @ V.T
    Y[:, 1::3] = Y[:, 0::3][:, : Y[:, 1::3].shape[1]] * 0.999 + 1e-3 * Y[:, 1::3]
    perm0, _, k = H.cpqr_eps(Y, 1e-3)
    assert 0 < k < m
    perm, W, swaps = H.strong_rrqr(Y, perm0, k, f)
    assert swaps < H.SRRQR_MAX_SWAPS
    ok, worst = _no_volume_gain_above(Y, list(perm[:k]), f)
    assert ok, worst
    X = np.linalg.solve(np.triu(W[:k, :k]), W[:k, k:])
    assert np.max(np.abs(X)) <= f * (1 + 1e-12)


def test_each_interchange_gains_more_than_f_in_volume():
    """Stopping after s interchanges for s = 0, 1, ...: s = 0 is the
    column-pivoted QR's selection, each further interchange multiplies the
    volume of the selection by more than f (Gu and Eisenstat's argument for
    termination), and the interchanges stop at the first selection from
    which no interchange gains more than f."""
    n, c, f = 20, 0.35, 1.5
    K = _kahan(n, c)
    perm0, _, _ = H.cpqr_eps(K, 1e-300)
    k = n - 2
    sels = []
    s = 0
    while True:
        perm, _, sw = H.strong_rrqr(K, perm0, k, f, max_swaps=s)
        sels.append(list(perm[:k]))
        if sw < s:
            break
        s += 1
    assert len(sels) >= 3
    assert sorted(sels[0]) == list(range(k))
    vols = [_logvol(K, J) for J in sels[:-1]]
    for a, b in zip(vols, vols[1:]):
        assert b - a > np.log(f)
    # it stops at the first selection that meets the bound: every earlier
    # one has an interchange gaining more than f (brute force), the last
    # has none
    for J in sels[:-2]:
        assert not _no_volume_gain_above(K, J, f, rel=-1e-9)[0]
    assert _no_volume_gain_above(K, sels[-1], f)[0]


def test_exact_rank_id_still_reconstructs():
    """For Y of exact rank r the ID with strong RRQR still reproduces Y
    from r of its columns: Y^T = Pi [I; E] Y[:, J]^T, and |E| <= f."""
    rg = np.random.default_rng(7)
    d, m, r, f = 30, 40, 6, 1.02
    Y = rg.standard_normal((d, r)) @ (rg.standard_normal((r, m)) * np.logspace(0, -3, m))
    st = {}
    perm, E, k = H.interp_decomp(Y, 1e-10, srrqr_f=f, stats=st)
    assert k == r
    U = H.interp_matrix(perm, E)
    assert np.linalg.norm(Y.T - U @ Y[:, perm[:k]].T) <= 1e-11 * np.linalg.norm(Y)
    assert np.max(np.abs(E)) <= f * (1 + 1e-12)
    assert "swaps" in st


def test_large_f_changes_nothing():
    """With f beyond any interpolation coefficient no interchange happens
    and the ID is the column-pivoted QR's, bit for bit."""
    rg = np.random.default_rng(3)
    Y = rg.standard_normal((15, 25)) @ np.diag(np.logspace(0, -8, 25))
    p0, E0, k0 = H.interp_decomp(Y, 1e-6)
    st = {}
    p1, E1, k1 = H.interp_decomp(Y, 1e-6, srrqr_f=1e300, stats=st)
    assert st["swaps"] == 0 and k0 == k1
    assert np.array_equal(p0, p1) and np.array_equal(E0, E1)


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_interchanges_start_exactly_above_f(seed):
    """The threshold is the volume gain itself: with g0 the largest gain of
    a single interchange from the column-pivoted QR's selection (brute
    force), f = 1.01 g0 leaves that selection unchanged and f = 0.99 g0
    makes at least one interchange."""
    rg = np.random.default_rng(seed)
    d, m = 14, 22
    r = min(d, m)
    U = np.linalg.qr(rg.standard_normal((d, r)))[0]
    V = np.linalg.qr(rg.standard_normal((m, r)))[0]
    Y = U @ np.diag(0.6 ** np.arange(r)) @ V.T
    Y[:, 1::3] = Y[:, 0::3][:, : Y[:, 1::3].shape[1]] * 0.999 + 1e-3 * Y[:, 1::3]
    perm0, _, k = H.cpqr_eps(Y, 1e-3)
    _, worst = _no_volume_gain_above(Y, list(perm0[:k]), 1.0)
    g0 = float(np.exp(worst))
    assert g0 > 1.02
    _, _, sw_hi = H.strong_rrqr(Y, perm0, k, 1.01 * g0)
    _, _, sw_lo = H.strong_rrqr(Y, perm0, k, 0.99 * g0)
    assert sw_hi == 0 and sw_lo >= 1
