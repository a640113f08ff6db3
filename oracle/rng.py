"""Keyed Gaussian generator for the random sampling matrix R (oracle side).

The paper fills R element by element with a pseudo-random engine seeded per
row by the global row index, so that the R of two sibling fronts agree on
shared rows and a parent can reuse them (Sec. 2.2.3, Sec. 4.3, Eq. Rmerge).
Here that property is obtained with a counter-based generator: entry (row, c)
is a pure function of (seed, original row id, column c), so every front that
contains a row sees the same value and the extend-merge of Eq. Rmerge holds
by construction.

Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written from its published definition.
  key     = (row id, low 32 bits of seed)
  counter = (column, high 32 bits of seed, 0, 0)
Output words (x0, x1) give u1 in (0, 1] with 53 bits, (x2, x3) give u2 in
[0, 1); z = sqrt(-2 ln u1) cos(2 pi u2) (Box-Muller).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of uint32 (broadcast)."""
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint32) for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3, k0, k1 = (v.copy() for v in (c0, c1, c2, c3, k0, k1))
    with np.errstate(over="ignore"):
        for r in range(10):
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if r < 9:
                k0 = k0 + W0
                k1 = k1 + W1
    return c0, c1, c2, c3


def gaussian(seed, rows, ncols, col0=0):
    """R[r, c] for r in ``rows`` (original row ids) and c in [col0, col0+ncols).
    Returns a float64 array of shape (len(rows), ncols)."""
    rows = np.asarray(rows, dtype=np.int64).reshape(-1, 1)
    cols = np.arange(col0, col0 + ncols, dtype=np.int64).reshape(1, -1)
    seed = int(seed)
    x0, x1, x2, x3 = philox4x32_10(cols.astype(np.uint32), np.uint32((seed >> 32) & 0xFFFFFFFF),
                                   np.uint32(0), np.uint32(0),
                                   rows.astype(np.uint32), np.uint32(seed & 0xFFFFFFFF))
    a = (x0 >> np.uint32(5)).astype(np.float64)
    b = (x1 >> np.uint32(6)).astype(np.float64)
    u1 = (a * 67108864.0 + b + 1.0) * (1.0 / 9007199254740992.0)
    a2 = (x2 >> np.uint32(5)).astype(np.float64)
    b2 = (x3 >> np.uint32(6)).astype(np.float64)
    u2 = (a2 * 67108864.0 + b2) * (1.0 / 9007199254740992.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
