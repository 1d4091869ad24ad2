"""Direct solves: banded LU with partial pivoting, and SuperLU.

Part of the CPU oracle (test infrastructure only).

The banded LU follows the usual band-Gaussian-elimination scheme (the
semantics of LAPACK's general band factorisation): unknowns are reordered to
shrink the half-bandwidth, the matrix is stored column by column with room
for the ``kl`` extra superdiagonals that row interchanges create, each
column is eliminated after swapping in its largest-magnitude candidate
pivot, and the multipliers stay in place as elementary transforms applied
in the forward substitution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import reverse_cuthill_mckee


def bandwidth(A):
    A = sp.coo_matrix(A)
    d = A.row.astype(np.int64) - A.col.astype(np.int64)
    return int(max(d.max(), 0)), int(max((-d).max(), 0))


def band_permutation(A, xyz=None):
    """Ordering that shrinks the half-bandwidth: reverse Cuthill-McKee on A's
    pattern, or, when node coordinates are given, the lexicographic
    coordinate orderings (each axis order tried), whichever is narrowest."""
    cands = [reverse_cuthill_mckee(sp.csr_matrix(A), symmetric_mode=True)]
    if xyz is not None:
        import itertools
        for order in itertools.permutations(range(3)):
            keys = tuple(np.round(xyz[:, d], 12) for d in order)   # last key is the primary one
            cands.append(np.lexsort(keys))
    best, bw = None, None
    for p in cands:
        Ap = sp.csr_matrix(A)[p][:, p]
        w = max(bandwidth(Ap))
        if bw is None or w < bw:
            best, bw = p, w
    return best


class BandedLU:
    """LU with partial pivoting of a (permuted) band matrix, complex128."""

    def __init__(self, A, perm=None):
        A = sp.csr_matrix(A, dtype=np.complex128)
        n = A.shape[0]
        self.perm = np.arange(n) if perm is None else np.asarray(perm)
        Ap = A[self.perm][:, self.perm].tocoo()
        kl, ku = bandwidth(Ap)
        kv = kl + ku
        ab = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128)
        ab[kv + Ap.row - Ap.col, Ap.col] = Ap.data
        ipiv = np.arange(n)
        ju = 0
        for j in range(n):
            km = min(kl, n - 1 - j)
            col = ab[kv:kv + km + 1, j]
            p = int(np.argmax(np.abs(col)))
            ipiv[j] = j + p
            ju = max(ju, min(j + ku + p, n - 1))
            if col[p] == 0:
                continue                      # exactly singular column: left as is
            cols = np.arange(j, ju + 1)
            if p != 0:
                r1 = kv + j - cols
                t = ab[r1, cols].copy()
                ab[r1, cols] = ab[r1 + p, cols]
                ab[r1 + p, cols] = t
            if km > 0:
                ab[kv + 1:kv + km + 1, j] /= ab[kv, j]
                if ju > j:
                    c = cols[1:]
                    i = np.arange(j + 1, j + km + 1)
                    R = kv + i[:, None] - c[None, :]
                    l = ab[kv + 1:kv + km + 1, j]
                    u = ab[kv + j - c, c]
                    ab[R, c[None, :]] -= l[:, None] * u[None, :]
        self.ab, self.ipiv, self.kl, self.ku, self.n = ab, ipiv, kl, ku, n

    def solve(self, b):
        ab, kl, ku, n = self.ab, self.kl, self.ku, self.n
        kv = kl + ku
        x = np.asarray(b, dtype=np.complex128)[self.perm].copy()
        for j in range(n - 1):
            km = min(kl, n - 1 - j)
            p = self.ipiv[j]
            if p != j:
                x[j], x[p] = x[p], x[j]
            x[j + 1:j + km + 1] -= ab[kv + 1:kv + km + 1, j] * x[j]
        for j in range(n - 1, -1, -1):
            x[j] /= ab[kv, j]
            i0 = max(0, j - kv)
            if j > i0:
                x[i0:j] -= ab[kv + i0 - j:kv, j] * x[j]
        out = np.empty_like(x)
        out[self.perm] = x
        return out


def banded_solve(A, f, xyz=None):
    """Solve A x = f by banded LU after a bandwidth-reducing reordering."""
    return BandedLU(A, band_permutation(A, xyz)).solve(f)


class SparseLU:
    """SuperLU factorisation (scipy) for meshes too large for the band code.
    ``ordering`` is SuperLU's fill-reducing column ordering (its default
    COLAMD, or e.g. ``"MMD_AT_PLUS_A"``, minimum degree on the symmetric
    pattern, which fills less on these 3-D meshes); it changes the rounding,
    not the factorisation's definition (LU with partial pivoting)."""

    def __init__(self, A, ordering=None):
        kw = {} if ordering is None else {"permc_spec": ordering}
        self.lu = spla.splu(sp.csc_matrix(A, dtype=np.complex128), **kw)

    def solve(self, b):
        return self.lu.solve(np.asarray(b, dtype=np.complex128))
