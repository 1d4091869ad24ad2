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
* The sun-roof forcing is a Neumann datum ``g`` on the roof patch,
  nodal-interpolated, so the load is ``f = Mpatch g`` (the default).
* Or, as the paper states it, a Dirichlet condition on the opening
  (``dirichlet=True``): the pressure is prescribed, ``p = g``, at every node
  of the source faces (set D; the paper's spectrum values are not available,
  synthetic nodal values stand in).  The condition is imposed by symmetric
  elimination: with F the other nodes, ``A_FF p_F = -A_FD g_D``, written as
  one system of the full size whose D rows and columns are those of the
  identity, ``A' p = f'`` with ``f'_F = -A_FD g_D`` and ``f'_D = g_D``
  (A' stays complex symmetric).
* The paper discretises with stabilised finite elements without giving the
  scheme.  ``gls=True`` takes the Galerkin least-squares method of Harari
  and Hughes for the Helmholtz operator (Comput. Methods Appl. Mech. Engrg.
  98, 1992): it adds ``tau (L w, L p)`` element by element with
  ``L = -lap - k^2``.  The Laplacian of a trilinear (or linear) shape
  function vanishes inside an element, so the added term is
  ``tau k^4 M``: the mass coefficient ``k^2`` becomes ``k^2 (1 - tau k^2)``.
  Their ``tau`` for linear elements makes the 1-D discrete dispersion
  relation exact: ``tau k^2 = 1 - 6 (1 - cos kh) / ((kh)^2 (2 + cos kh))``;
  ``h`` is taken as the mean element edge length of the mesh (one value for
  the mesh, exact for the uniform boxes here).  The absorption term keeps
  ``k^2``.

So ``A(k) = K - m(k) M + i k^2 M_eta + i k B_beta`` with ``m(k) = k^2``
(Galerkin) or ``k^2 (1 - tau k^2)`` (GLS), complex symmetric, and
``A(k) p = f``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def gls_tau_k2(kh):
    """Harari-Hughes GLS parameter ``tau k^2`` of linear elements of size h
    at wavenumber k (``1 - 6 (1 - cos kh) / ((kh)^2 (2 + cos kh))``; its
    small-kh limit is ``-(kh)^2 / 12``)."""
    t = float(kh)
    if t == 0.0:
        return 0.0
    return 1.0 - 6.0 * (1.0 - np.cos(t)) / (t * t * (2.0 + np.cos(t)))


def mean_edge_length(mesh):
    """Mean length of the element edges (hexahedra: the 12 pairs of tensor
    corners differing in one index; tetrahedra: the 6 vertex pairs)."""
    el = fem.elements(mesh)
    xyz = mesh["xyz"]
    if el.shape[1] == 8:
        pairs = [(a, a | b) for b in (1, 2, 4) for a in range(8) if not a & b]
    else:
        pairs = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    lens = [np.linalg.norm(xyz[el[:, a]] - xyz[el[:, b]], axis=1) for a, b in pairs]
    return float(np.mean(np.stack(lens)))


def dirichlet_nodes(mesh):
    """Sorted ids of the nodes of the source faces (the Dirichlet set D)."""
    return np.unique(mesh["bface"][mesh["bface_src"] == 1].ravel()).astype(np.int64)


class System:
    """Assembled real parts of one mesh plus the complex parameters.
    ``dirichlet``: prescribe p on the source faces' nodes instead of a
    Neumann datum; ``gls``: Galerkin least-squares mass coefficient."""

    def __init__(self, mesh, beta, eta=None, dirichlet=False, gls=False):
        self.mesh = mesh
        self.asm = fem.assemble(mesh, with_element_mass=eta is not None)
        self.n = mesh["xyz"].shape[0]
        self.dirichlet = bool(dirichlet)
        self.D = dirichlet_nodes(mesh) if self.dirichlet else np.zeros(0, dtype=np.int64)
        self.gls_h = mean_edge_length(mesh) if gls else 0.0
        self.set_params(beta, eta)

    def mass_coefficient(self, k):
        """m(k): k^2, or k^2 (1 - tau k^2) with the GLS tau."""
        if self.gls_h == 0.0:
            return k * k
        return k * k * (1.0 - gls_tau_k2(k * self.gls_h))

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

    def operator(self, k, eliminate=True):
        """A(k) as a complex128 CSR matrix; with a Dirichlet set (and
        eliminate) the rows and columns of D replaced by the identity's."""
        K, M = self.asm["K"], self.asm["M"]
        A = K.astype(np.complex128) - self.mass_coefficient(k) * M + (1j * k) * self.Bbeta
        if self.Meta is not None:
            A = A + (1j * k * k) * self.Meta
        if self.dirichlet and eliminate:
            keep = np.ones(self.n)
            keep[self.D] = 0.0
            Pf = sp.diags(keep)
            A = Pf @ A @ Pf + sp.diags(1.0 - keep)
        A = sp.csr_matrix(A)
        if self.dirichlet and eliminate:
            A.eliminate_zeros()
        A.sort_indices()
        return A

    def load(self, g, k=None):
        """Neumann: f = Mpatch g (g: nodal amplitudes on the roof patch).
        Dirichlet (needs k): f'_F = -A_FD g_D, f'_D = g_D."""
        g = np.asarray(g, dtype=np.complex128)
        if not self.dirichlet:
            return self.asm["Mpatch"] @ g
        if k is None:
            raise ValueError("the Dirichlet load depends on the frequency: pass k")
        gD = np.zeros(self.n, dtype=np.complex128)
        gD[self.D] = g[self.D]
        f = -(self.operator(k, eliminate=False) @ gD)
        f[self.D] = g[self.D]
        return f


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
