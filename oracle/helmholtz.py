"""The discrete Helmholtz operator and load.

Part of the CPU oracle (test infrastructure only).

Paper Sec. 3.2: Fourier-transforming the homogeneous wave equation gives the
Helmholtz equation ``-w^2 psi - c^2 lap(psi) = 0``, i.e. ``-lap(p) - k^2 p = 0``
with ``k = w / c``.  The readings taken where the paper is silent:

* Walls carry a Robin (impedance) condition ``dp/dn + i k beta_w p = g`` with
  ``beta_w`` the normalised outward admittance of wall ``w``; ``Re beta >= 0``
  absorbs.  This gives the boundary term ``+ i k sum_w beta_w B0_w``.
* An optional per-element loss factor ``eta_e`` turns the element's ``k^2``
  into ``k^2 (1 - i eta_e)``, i.e. the term ``+ i k^2 sum_e eta_e M_e``.
* The sun-roof forcing is a Neumann datum ``g`` on the roof patch (the paper's
  Dirichlet spectrum data is not available), nodal-interpolated, so the load
  is ``f = Mpatch g``.

So ``A(k) = K - k^2 M + i k^2 M_eta + i k B_beta`` (complex symmetric) and
``A(k) p = f``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


class System:
    """Assembled real parts of one mesh plus the complex parameters."""

    def __init__(self, mesh, beta, eta=None):
        self.mesh = mesh
        self.asm = fem.assemble(mesh, with_element_mass=eta is not None)
        self.n = mesh["xyz"].shape[0]
        self.set_params(beta, eta)

    def set_params(self, beta, eta=None):
        self.beta = np.asarray(beta, dtype=np.complex128).copy()
        self.Bbeta = sum(self.beta[w] * self.asm["B0"][w] for w in range(6))
        self.eta = None if eta is None else np.asarray(eta, dtype=np.float64).copy()
        if self.eta is not None:
            if "Me" not in self.asm:
                self.asm = fem.assemble(self.mesh, with_element_mass=True)
            self.Meta = fem.element_weighted_mass(self.mesh, self.asm["Me"], self.eta)
        else:
            self.Meta = None

    def operator(self, k):
        """A(k) as a complex128 CSR matrix."""
        K, M = self.asm["K"], self.asm["M"]
        A = K.astype(np.complex128) - (k * k) * M + (1j * k) * self.Bbeta
        if self.Meta is not None:
            A = A + (1j * k * k) * self.Meta
        A = sp.csr_matrix(A)
        A.sort_indices()
        return A

    def load(self, g):
        """f = Mpatch g (g: nodal Neumann amplitudes on the roof patch)."""
        return self.asm["Mpatch"] @ np.asarray(g, dtype=np.complex128)


def relres(A, x, f):
    """True relative residual ``||f - A x||_2 / ||f||_2`` in complex128."""
    return np.linalg.norm(f - A @ x) / np.linalg.norm(f)


def apply_elementwise(mesh, k, beta, eta, x, chunk=200_000):
    """Matrix-free ``y = A(k) x`` summed element by element (no CSR), used to
    check residuals at sizes where building the CSR on the CPU is slow."""
    xyz = mesh["xyz"]
    hexes = fem.elements(mesh)
    n = xyz.shape[0]
    x = np.asarray(x, dtype=np.complex128)
    yr = np.zeros(n)
    yi = np.zeros(n)
    for s in range(0, hexes.shape[0], chunk):
        h = hexes[s:s + chunk]
        Ke, Me = fem.element_matrices(xyz[h])
        Ae = Ke.astype(np.complex128) - (k * k) * Me
        if eta is not None:
            Ae = Ae + (1j * k * k) * np.asarray(eta[s:s + chunk])[:, None, None] * Me
        ye = np.einsum("eab,eb->ea", Ae, x[h])
        yr += np.bincount(h.ravel(), weights=ye.real.ravel(), minlength=n)
        yi += np.bincount(h.ravel(), weights=ye.imag.ravel(), minlength=n)
    bf = mesh["bface"].astype(np.int64)
    tag = mesh["bface_tag"]
    for s in range(0, bf.shape[0], chunk):
        q = bf[s:s + chunk]
        Fe = fem.face_mass(xyz[q]).astype(np.complex128)
        Fe *= (1j * k * np.asarray(beta, dtype=np.complex128)[tag[s:s + chunk]])[:, None, None]
        ye = np.einsum("eab,eb->ea", Fe, x[q])
        yr += np.bincount(q.ravel(), weights=ye.real.ravel(), minlength=n)
        yi += np.bincount(q.ravel(), weights=ye.imag.ravel(), minlength=n)
    return yr + 1j * yi


def load_elementwise(mesh, g):
    """f = Mpatch g summed face by face (matrix-free)."""
    xyz = mesh["xyz"]
    bf = mesh["bface"][mesh["bface_src"] == 1].astype(np.int64)
    n = xyz.shape[0]
    Fe = fem.face_mass(xyz[bf])
    ye = np.einsum("eab,eb->ea", Fe, np.asarray(g, dtype=np.complex128)[bf])
    return (np.bincount(bf.ravel(), weights=ye.real.ravel(), minlength=n)
            + 1j * np.bincount(bf.ravel(), weights=ye.imag.ravel(), minlength=n))


def rows_of_operator(mesh, k, beta, eta, rows):
    """Selected rows of A(k), computed only from the elements and faces that
    touch them: returns a CSR matrix of shape (len(rows), n)."""
    rows = np.asarray(rows, dtype=np.int64)
    xyz = mesh["xyz"]
    n = xyz.shape[0]
    pos = -np.ones(n, dtype=np.int64)
    pos[rows] = np.arange(rows.size)
    hexes = fem.elements(mesh)
    esel = np.flatnonzero((pos[hexes] >= 0).any(axis=1))
    h = hexes[esel]
    npe = h.shape[1]
    Ke, Me = fem.element_matrices(xyz[h])
    Ae = Ke.astype(np.complex128) - (k * k) * Me
    if eta is not None:
        Ae = Ae + (1j * k * k) * np.asarray(eta)[esel][:, None, None] * Me
    r = np.repeat(h, npe, axis=1).ravel()
    c = np.tile(h, (1, npe)).ravel()
    v = Ae.reshape(-1)
    bf = mesh["bface"].astype(np.int64)
    fsel = np.flatnonzero((pos[bf] >= 0).any(axis=1))
    q = bf[fsel]
    npf = q.shape[1]
    Fe = fem.face_mass(xyz[q]).astype(np.complex128)
    Fe *= (1j * k * np.asarray(beta)[mesh["bface_tag"][fsel]])[:, None, None]
    r = np.concatenate([r, np.repeat(q, npf, axis=1).ravel()])
    c = np.concatenate([c, np.tile(q, (1, npf)).ravel()])
    v = np.concatenate([v, Fe.reshape(-1)])
    keep = pos[r] >= 0
    return sp.csr_matrix((v[keep], (pos[r[keep]], c[keep])), shape=(rows.size, n))
