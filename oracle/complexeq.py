"""Complex systems through their real-equivalent form (oracle side; test
infrastructure only, like the rest of this package).

The Helmholtz problems of Sec. 6.1 are complex.  A complex system A z = s is
equivalent to the real system of twice the size in which complex unknown j
becomes real unknowns 2j (real part) and 2j + 1 (imaginary part) and each
entry a + ib becomes the 2 x 2 block [a -b; b a]: (a + ib)(x + iy) =
(ax - by) + i(bx + ay).  The oracle's multifrontal method then runs on that
real system unchanged.  The block of the conjugate a - ib is the transpose
of the block of a + ib, so the real form's transpose is the real form of
A^H."""
import numpy as np

from paper_1502_07405_amd.problems import CSR, Ordering


def real_form(A):
    """The real-equivalent CSR (2n unknowns) of a complex CSR ``A``
    (problems.ZCSR): entry (i, j) = a + ib gives entries (2i, 2j) = a,
    (2i, 2j+1) = -b, (2i+1, 2j) = b, (2i+1, 2j+1) = a."""
    n = A.n
    rows, cols, vals = [], [], []
    for i in range(n):
        for e in range(A.rowptr[i], A.rowptr[i + 1]):
            j = int(A.colind[e])
            a, b = A.val[e].real, A.val[e].imag
            rows += [2 * i, 2 * i, 2 * i + 1, 2 * i + 1]
            cols += [2 * j, 2 * j + 1, 2 * j, 2 * j + 1]
            vals += [a, -b, b, a]
    rows = np.array(rows)
    cols = np.array(cols)
    vals = np.array(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rowptr = np.zeros(2 * n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return CSR(2 * n, np.cumsum(rowptr), cols[order].astype(np.int32), vals[order])


def real_ordering(o):
    """The ordering of the real form: each complex unknown's pair stays
    together, in the complex ordering's place (separators twice as long)."""
    perm = np.empty(2 * len(o.perm), dtype=np.int32)
    perm[0::2] = 2 * np.asarray(o.perm)
    perm[1::2] = 2 * np.asarray(o.perm) + 1
    return Ordering(perm, 2 * np.asarray(o.sep_ptr, dtype=np.int32), np.asarray(o.parent, dtype=np.int32),
                    o.boxes, o.dims)


def to_real(z):
    """A complex vector as the real form's vector (interleaved parts)."""
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(2 * z.shape[0])
    out[0::2] = z.real
    out[1::2] = z.imag
    return out


def to_complex(x):
    x = np.asarray(x, dtype=np.float64)
    return x[0::2] + 1j * x[1::2]
