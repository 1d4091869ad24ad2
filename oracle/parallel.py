"""Row-block threaded sparse product, for timing the oracle on all host cores.

TEST AND MEASUREMENT INFRASTRUCTURE ONLY, like the rest of this package.

The rows of a CSR matrix are cut into contiguous blocks, one per thread, and
each block's product is SciPy's own CSR routine (which releases the GIL), so
every entry of ``y = A @ x`` is the same sum in the same order as the
single-threaded product: the results are bitwise equal, and an oracle solver
given this operator takes exactly the same iterates.  The solvers only need
``@``, ``shape`` and ``diagonal()``.
"""
from __future__ import annotations

import concurrent.futures as cf

import numpy as np
import scipy.sparse as sp


class RowBlockOperator:
    def __init__(self, A, threads):
        self.A = sp.csr_matrix(A)
        self.shape = self.A.shape
        self.dtype = self.A.dtype
        self.threads = max(1, int(threads))
        n = self.shape[0]
        # blocks of about equal nonzero counts
        nnz_cut = np.linspace(0, self.A.nnz, self.threads + 1)
        cuts = np.searchsorted(self.A.indptr, nnz_cut).clip(0, n)
        cuts[0], cuts[-1] = 0, n
        self.cuts = np.maximum.accumulate(cuts)
        self.blocks = [self.A[self.cuts[i]:self.cuts[i + 1]] for i in range(self.threads)]
        self.pool = cf.ThreadPoolExecutor(self.threads)

    def diagonal(self):
        return self.A.diagonal()

    def __matmul__(self, x):
        out = np.empty(self.shape[0], dtype=np.result_type(self.dtype, np.asarray(x).dtype))

        def one(i):
            out[self.cuts[i]:self.cuts[i + 1]] = self.blocks[i] @ x

        list(self.pool.map(one, range(self.threads)))
        return out

    def close(self):
        self.pool.shutdown()
