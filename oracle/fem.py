"""Q1 (trilinear hexahedron) and P1 (linear tetrahedron) Galerkin matrices
for the Helmholtz weak form.

Part of the CPU oracle (test infrastructure only).

The paper discretises the Helmholtz equation of Sec. 3.2 by finite elements
on the compartment mesh.  Its stabilised scheme is not given, so the oracle
uses plain Galerkin Q1 elements.  Multiplying ``-lap(p) - k^2 p = 0`` by a
test function and integrating by parts gives the bilinear forms

    K_ab = int grad(phi_a) . grad(phi_b),   M_ab = int phi_a phi_b,
    B0_w,ab = int_{wall w} phi_a phi_b,

with ``phi`` the trilinear shape functions.  Integrals use 2x2x2 (cells) and
2x2 (faces) Gauss-Legendre points, exact for Q1 on parallelepipeds.

Local node ``a`` of a hexahedron sits at reference corner
``(2*bit0(a)-1, 2*bit1(a)-1, 2*bit2(a)-1)``; of a quad at
``(2*bit0(a)-1, 2*bit1(a)-1)``.

A tetrahedral mesh (key ``tet``, 4 nodes per element, triangles as boundary
faces) uses P1 elements: the shape functions are the barycentric
coordinates, whose gradients are constant, so every integral is a closed
form (no quadrature): ``K_ab = V grad(l_a).grad(l_b)``,
``M_ab = V (1 + delta_ab) / 20``, face ``F_ab = A (1 + delta_ab) / 12``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

GAUSS = (-1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0))   # 2-point rule, weights 1


def _corner_signs(ndim):
    n = 2 ** ndim
    return np.array([[2 * ((a >> d) & 1) - 1 for d in range(ndim)] for a in range(n)],
                    dtype=np.float64)


def shape_hex(xi):
    """Trilinear shape functions at reference point ``xi`` (3,).

    Returns ``N`` (8,) and ``dN`` (8,3) = dN_a/dxi_d."""
    s = _corner_signs(3)
    f = 1.0 + s * np.asarray(xi)[None, :]          # (8,3) factors (1 + s_d xi_d)
    N = np.prod(f, axis=1) / 8.0
    dN = np.empty((8, 3))
    for d in range(3):
        others = [e for e in range(3) if e != d]
        dN[:, d] = s[:, d] * f[:, others[0]] * f[:, others[1]] / 8.0
    return N, dN


def shape_quad(xi):
    """Bilinear shape functions on the reference square: ``N`` (4,), ``dN`` (4,2)."""
    s = _corner_signs(2)
    f = 1.0 + s * np.asarray(xi)[None, :]
    N = f[:, 0] * f[:, 1] / 4.0
    dN = np.stack([s[:, 0] * f[:, 1], s[:, 1] * f[:, 0]], axis=1) / 4.0
    return N, dN


def hex_matrices(X):
    """Element stiffness and mass matrices of trilinear hexahedra.

    ``X`` (ne,8,3) corner coordinates in local order.  Returns ``Ke``, ``Me``
    (ne,8,8), each made exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    ne = X.shape[0]
    Ke = np.zeros((ne, 8, 8))
    Me = np.zeros((ne, 8, 8))
    for gz in GAUSS:
        for gy in GAUSS:
            for gx in GAUSS:
                N, dN = shape_hex((gx, gy, gz))
                J = np.einsum("eai,ad->eid", X, dN)          # dx_i/dxi_d
                detJ = np.linalg.det(J)
                Jinv = np.linalg.inv(J)                       # dxi_d/dx_i
                G = np.einsum("ad,edi->eai", dN, Jinv)        # grad phi_a
                Ke += np.einsum("eai,ebi->eab", G, G) * detJ[:, None, None]
                Me += np.outer(N, N)[None] * detJ[:, None, None]
    Ke = 0.5 * (Ke + Ke.transpose(0, 2, 1))
    Me = 0.5 * (Me + Me.transpose(0, 2, 1))
    return Ke, Me


def quad_mass(X):
    """Boundary-face mass matrices ``int_face phi_a phi_b`` of bilinear quads
    embedded in 3-D.  ``X`` (nf,4,3) -> (nf,4,4), exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    nf = X.shape[0]
    Fe = np.zeros((nf, 4, 4))
    for gy in GAUSS:
        for gx in GAUSS:
            N, dN = shape_quad((gx, gy))
            t = np.einsum("eai,ad->edi", X, dN)              # two tangents
            area = np.linalg.norm(np.cross(t[:, 0], t[:, 1]), axis=1)
            Fe += np.outer(N, N)[None] * area[:, None, None]
    return 0.5 * (Fe + Fe.transpose(0, 2, 1))


def tet_matrices(X):
    """Element stiffness and mass matrices of linear tetrahedra (closed forms).

    ``X`` (ne,4,3) vertex coordinates.  With ``D`` the edge matrix (columns
    ``x_a - x_0``, a = 1..3), the barycentric gradients of vertices 1..3 are
    the rows of ``D^-1`` and that of vertex 0 is minus their sum; the volume
    is ``|det D| / 6``.  Returns ``Ke``, ``Me`` (ne,4,4), exactly symmetric."""
    X = np.asarray(X, dtype=np.float64)
    D = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)   # columns
    vol = np.abs(np.linalg.det(D)) / 6.0
    Dinv = np.linalg.inv(D)
    G = np.concatenate([-Dinv.sum(axis=1, keepdims=True), Dinv], axis=1)             # (ne,4,3)
    Ke = np.einsum("eai,ebi->eab", G, G) * vol[:, None, None]
    Me = (np.ones((4, 4)) + np.eye(4))[None] * (vol / 20.0)[:, None, None]
    Ke = 0.5 * (Ke + Ke.transpose(0, 2, 1))
    return Ke, Me


def tri_mass(X):
    """Boundary-face mass ``int_face phi_a phi_b`` of linear triangles:
    ``A (1 + delta_ab) / 12`` with ``A`` the area.  ``X`` (nf,3,3)."""
    X = np.asarray(X, dtype=np.float64)
    area = 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1)
    return (np.ones((3, 3)) + np.eye(3))[None] * (area / 12.0)[:, None, None]


def elements(mesh):
    """Element connectivity (int64) of a hexahedral (``hex``) or tetrahedral
    (``tet``) mesh."""
    conn = mesh["tet"] if "tet" in mesh else mesh["hex"]
    return np.asarray(conn, dtype=np.int64)


def element_matrices(X):
    """``Ke``, ``Me`` of Q1 hexahedra (8 nodes) or P1 tetrahedra (4 nodes)."""
    return tet_matrices(X) if X.shape[1] == 4 else hex_matrices(X)


def face_mass(X):
    """Boundary-face mass of bilinear quads (4 nodes) or linear triangles (3)."""
    return tri_mass(X) if X.shape[1] == 3 else quad_mass(X)


class Pattern:
    """COO -> CSR summation in a fixed order.

    Entries are stably sorted by (row, col) and duplicates are summed in
    their original (element) order, so the (i,j) and (j,i) entries of a
    matrix assembled from symmetric element matrices are summed from the
    same terms in the same order: the result is bitwise symmetric."""

    def __init__(self, conn, n):
        conn = np.asarray(conn, dtype=np.int64)
        nloc = conn.shape[1]
        rows = np.repeat(conn, nloc, axis=1).ravel()
        cols = np.tile(conn, (1, nloc)).ravel()
        key = rows * n + cols
        self.order = np.argsort(key, kind="stable")
        ks = key[self.order]
        first = np.ones(ks.size, dtype=bool)
        first[1:] = ks[1:] != ks[:-1]
        self.starts = np.flatnonzero(first)
        uk = ks[self.starts]
        self.n = n
        self.indices = (uk % n).astype(np.int64)
        r = uk // n
        self.indptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(self.indptr, r + 1, 1)
        self.indptr = np.cumsum(self.indptr)

    def matrix(self, elem_vals):
        v = np.asarray(elem_vals).reshape(-1)[self.order]
        data = np.add.reduceat(v, self.starts)
        return sp.csr_matrix((data, self.indices.copy(), self.indptr.copy()),
                             shape=(self.n, self.n))


def assemble(mesh, with_element_mass=False):
    """Assemble the real matrices of a hexahedral (Q1) or tetrahedral (P1) mesh.

    Returns a dict of scipy CSR matrices over the full cell pattern:
    ``K``, ``M``, ``B0`` (list of 6, wall w = tag w), ``Mpatch`` (faces with
    the source flag), and, on request, the element mass array ``Me``
    (ne,8,8) or (ne,4,4) used for the absorption field."""
    xyz = mesh["xyz"]
    conn = elements(mesh)
    n = xyz.shape[0]
    Ke, Me = element_matrices(xyz[conn])
    pat = Pattern(conn, n)
    out = dict(K=pat.matrix(Ke), M=pat.matrix(Me), pattern=pat)
    bf = mesh["bface"].astype(np.int64)
    Fe = face_mass(xyz[bf])
    out["B0"] = []
    for w in range(6):
        sel = mesh["bface_tag"] == w
        out["B0"].append(_face_matrix(bf[sel], Fe[sel], n))
    sel = mesh["bface_src"] == 1
    out["Mpatch"] = _face_matrix(bf[sel], Fe[sel], n)
    if with_element_mass:
        out["Me"] = Me
    return out


def _face_matrix(faces, Fe, n):
    if faces.shape[0] == 0:
        return sp.csr_matrix((n, n))
    return Pattern(faces, n).matrix(Fe)


def element_weighted_mass(mesh, Me, weights):
    """``sum_e w_e M_e`` assembled on the cell pattern (w = absorption field)."""
    pat = Pattern(elements(mesh), mesh["xyz"].shape[0])
    return pat.matrix(Me * np.asarray(weights, dtype=np.float64)[:, None, None])
