"""Pins of the oracle's finite-element assembly against closed forms.

Each check here comes from the mathematics of Q1 elements on a box, not from
the oracle itself: Kronecker closed forms of the element matrices, the exact
discrete eigenvectors of the rigid box, an exact 1-D reduction of the full
3-D solve, and the O(h^2) convergence to a manufactured plane wave.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import direct, fem, helmholtz as H

pytestmark = pytest.mark.cpu


def M1(h):
    return (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])


def K1(h):
    return (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])


def test_p1_element_matrices_closed_form():
    hx, hy, hz = 0.37, 0.21, 0.55
    X = np.array([[[a * hx, b * hy, c * hz] for c in range(2) for b in range(2) for a in range(2)]],
                 dtype=float)
    # reorder to local index a + 2b + 4c
    X = np.array([[[((i >> 0) & 1) * hx, ((i >> 1) & 1) * hy, ((i >> 2) & 1) * hz] for i in range(8)]])
    Ke, Me = fem.hex_matrices(X + np.array([0.3, -1.1, 2.0]))
    Mref = np.kron(M1(hz), np.kron(M1(hy), M1(hx)))
    Kref = (np.kron(M1(hz), np.kron(M1(hy), K1(hx))) + np.kron(M1(hz), np.kron(K1(hy), M1(hx)))
            + np.kron(K1(hz), np.kron(M1(hy), M1(hx))))
    assert np.allclose(Me[0], Mref, rtol=1e-15, atol=1e-15 * abs(Mref).max())
    assert np.allclose(Ke[0], Kref, rtol=1e-14, atol=1e-14 * abs(Kref).max())
    # a face in the y-z plane (x = const): in-plane axes y (fast), z
    Xf = np.array([[[0.7, ((i >> 0) & 1) * hy, ((i >> 1) & 1) * hz] for i in range(4)]])
    Fe = fem.quad_mass(Xf)
    assert np.allclose(Fe[0], np.kron(M1(hz), M1(hy)), rtol=1e-15, atol=1e-16)


def test_p1_element_matrices_affine_rotation_invariant():
    # mass and stiffness of a rotated box element equal those of the unrotated one
    hx, hy, hz = 0.2, 0.3, 0.4
    X = np.array([[((i >> 0) & 1) * hx, ((i >> 1) & 1) * hy, ((i >> 2) & 1) * hz] for i in range(8)])
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    K0, M0 = fem.hex_matrices(X[None])
    K1_, M1_ = fem.hex_matrices((X @ R.T)[None])
    assert np.allclose(K0, K1_, atol=1e-13)
    assert np.allclose(M0, M1_, atol=1e-15)


@pytest.mark.parametrize("elems", [(20, 12, 10), (5, 3, 4)])
def test_p2_assembly_invariants(elems):
    mesh = W.box_mesh(*elems)
    asm = fem.assemble(mesh)
    K, M = asm["K"], asm["M"]
    for Mat in [K, M, asm["Mpatch"]] + asm["B0"]:
        assert (Mat != Mat.T).nnz == 0           # bitwise symmetric
    ones = np.ones(mesh["n_nodes"])
    assert np.abs(K @ ones).max() <= 1e-14 * np.abs(K.data).max()
    assert abs(M.sum() - 1.8 * 1.2 * 1.0) < 1e-12
    areas = [1.2, 1.2, 1.8, 1.8, 2.16, 2.16]
    for w in range(6):
        assert abs(asm["B0"][w].sum() - areas[w]) < 1e-12
    nx, ny, nz = elems
    assert K.nnz == (3 * nx + 1) * (3 * ny + 1) * (3 * nz + 1)
    # source patch: quads whose centroid lies in [0.6,1.2] x [0.3,0.9]
    hx, hy = 1.8 / nx, 1.2 / ny
    cx = (np.arange(nx) + 0.5) * hx
    cy = (np.arange(ny) + 0.5) * hy
    area = (((cx >= 0.6) & (cx <= 1.2)).sum() * hx) * (((cy >= 0.3) & (cy <= 0.9)).sum() * hy)
    assert abs(asm["Mpatch"].sum() - area) < 1e-12


def test_p2_patch_sizes_of_workloads():
    m = W.box_mesh(20, 12, 10)
    assert W.patch_nodes(m).size == 49
    asm = fem.assemble(m)
    assert abs(asm["Mpatch"].sum() - 0.54 * 0.60) < 1e-12
    m2 = W.box_mesh(80, 48, 40)
    assert W.patch_nodes(m2).size == 675


@pytest.mark.parametrize("elems,modes", [((20, 12, 10), [(1, 0, 0), (0, 1, 0), (2, 1, 3)]),
                                         ((7, 5, 3), [(1, 1, 1), (3, 0, 2)])])
def test_p3_discrete_rigid_box_modes(elems, modes):
    mesh = W.box_mesh(*elems)
    asm = fem.assemble(mesh)
    K, M = asm["K"], asm["M"]
    h = mesh["h"]
    for m in modes:
        vecs, lam = [], 0.0
        for d in range(3):
            N = elems[d]
            th = m[d] * np.pi / N
            vecs.append(np.cos(th * np.arange(N + 1)))
            lam += (6.0 / h[d] ** 2) * (1.0 - np.cos(th)) / (2.0 + np.cos(th))
        v = np.kron(vecs[2], np.kron(vecs[1], vecs[0]))
        Kv, Mv = K @ v, M @ v
        assert np.linalg.norm(Kv - lam * Mv) <= 1e-12 * max(np.linalg.norm(Kv), np.linalg.norm(lam * Mv), 1e-300) + 1e-13


def test_p3_first_mode_frequency_c0():
    # discrete (1,0,0) mode of the 20x12x10 mesh: 94.54 Hz vs continuum 94.44 Hz
    h = 1.8 / 20
    th = np.pi / 20
    lam = (6.0 / h ** 2) * (1 - np.cos(th)) / (2 + np.cos(th))
    f = 340.0 * np.sqrt(lam) / (2 * np.pi)
    assert abs(f - 94.54) < 0.01
    assert abs(340.0 / (2 * 1.8) - 94.444) < 1e-3


def _one_d_exact(N, h, k, g0, beta_xplus):
    """Exact nodal solution of the 1-D Q1 problem (K - k^2 M + i k beta e_N e_N^T) p = g0 e_0,
    built from the closed-form interior recurrence p_j = a cos(th (N-j)) + b sin(th (N-j))."""
    a2 = (k * h) ** 2
    th = np.arccos((1.0 - a2 / 3.0) / (1.0 + a2 / 6.0))
    j = np.arange(N + 1)
    C = np.cos(th * (N - j)).astype(complex)
    S = np.sin(th * (N - j)).astype(complex)

    def row0(v):
        return (v[0] - v[1]) / h - k * k * h / 6.0 * (2 * v[0] + v[1])

    def rowN(v):
        return (v[N] - v[N - 1]) / h - k * k * h / 6.0 * (2 * v[N] + v[N - 1]) + 1j * k * beta_xplus * v[N]

    Msys = np.array([[row0(C), row0(S)], [rowN(C), rowN(S)]])
    ab = np.linalg.solve(Msys, np.array([g0, 0.0], dtype=complex))
    return ab[0] * C + ab[1] * S


@pytest.mark.parametrize("beta_xplus", [0.0, 0.3 + 0.1j])
def test_p4_exact_one_d_reduction(beta_xplus):
    nx, ny, nz = 12, 3, 2
    mesh = W.box_mesh(nx, ny, nz)
    beta = np.zeros(6, dtype=complex)
    beta[1] = beta_xplus
    S = H.System(mesh, beta)
    k = W.wavenumber(120.0)
    A = S.operator(k)
    g0 = 0.7 - 0.4j
    f = S.asm["B0"][0] @ np.full(mesh["n_nodes"], g0)
    p = direct.SparseLU(A).solve(f)
    exact = _one_d_exact(nx, 1.8 / nx, k, g0, beta_xplus)
    i = np.arange(mesh["n_nodes"]) % (nx + 1)
    assert np.abs(p - exact[i]).max() <= 1e-10 * np.abs(exact).max()
    pb = direct.banded_solve(A, f, mesh["xyz"])
    assert np.abs(pb - exact[i]).max() <= 1e-10 * np.abs(exact).max()


def test_p5_manufactured_plane_wave_second_order():
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    k = W.wavenumber(200.0)
    beta = np.array([0.5, 0.4 + 0.1j, 0.3, 0.2 - 0.05j, 0.6, 0.45])
    normals = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    errs = []
    for lev in range(3):
        s = 2 ** lev
        mesh = W.box_mesh(9 * s, 6 * s, 5 * s)
        S = H.System(mesh, beta)
        pex = np.exp(-1j * k * (mesh["xyz"] @ d))
        f = np.zeros(mesh["n_nodes"], dtype=complex)
        for w in range(6):
            # dp/dn + i k beta p = g on wall w, with dp/dn = -i k (d.n) p
            gw = 1j * k * (beta[w] - d @ np.array(normals[w], float)) * pex
            f += S.asm["B0"][w] @ gw
        p = direct.SparseLU(S.operator(k)).solve(f)
        errs.append(np.abs(p - pex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.2), (errs, rates)


# ---------------------------------------------------------------- unstructured
@pytest.mark.parametrize("cells", [(3, 2, 2), (5, 4, 3)])
def test_p6_unstructured_mesh_invariants(cells):
    """Exact invariants of the assembly on the unstructured mesh (distorted,
    non-affine hexahedra, random node ids): total mass = box volume, wall
    masses = wall areas, constants in the kernel of K, and the patch test:
    trilinear elements reproduce a linear field exactly, so K u vanishes on
    every interior row for linear u."""
    mesh = W.kuhn_hex_mesh(*cells)
    asm = fem.assemble(mesh)
    K, M = asm["K"], asm["M"]
    n = mesh["n_nodes"]
    Lx, Ly, Lz = W.BOX
    assert abs(M.sum() - Lx * Ly * Lz) <= 1e-13
    areas = [Ly * Lz, Ly * Lz, Lx * Lz, Lx * Lz, Lx * Ly, Lx * Ly]
    for w in range(6):
        assert abs(asm["B0"][w].sum() - areas[w]) <= 1e-13
    assert abs(K - K.T).max() == 0.0 and abs(M - M.T).max() == 0.0
    assert np.abs(K @ np.ones(n)).max() <= 1e-13
    x = mesh["xyz"]
    u = 0.3 * x[:, 0] - 1.2 * x[:, 1] + 0.7 * x[:, 2] + 0.1
    r = K @ u
    wall = np.unique(mesh["bface"].ravel())
    inner = np.setdiff1d(np.arange(n), wall)
    assert inner.size > 0
    assert np.abs(r[inner]).max() <= 1e-13 * np.abs(r).max()


def test_p6_unstructured_plane_wave_second_order():
    """O(h^2) convergence to a plane wave with matching Robin data on
    unstructured meshes refined by halving the Kuhn cells."""
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    k = W.wavenumber(200.0)
    beta = np.array([0.5, 0.4 + 0.1j, 0.3, 0.2 - 0.05j, 0.6, 0.45])
    normals = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    errs = []
    for lev in range(3):
        s = 2 ** lev
        mesh = W.kuhn_hex_mesh(3 * s, 2 * s, 2 * s, jitter=0.0)
        S = H.System(mesh, beta)
        pex = np.exp(-1j * k * (mesh["xyz"] @ d))
        f = np.zeros(mesh["n_nodes"], dtype=complex)
        for w in range(6):
            gw = 1j * k * (beta[w] - d @ np.array(normals[w], float)) * pex
            f += S.asm["B0"][w] @ gw
        p = direct.SparseLU(S.operator(k)).solve(f)
        errs.append(np.abs(p - pex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.3), (errs, rates)


# ---------------------------------------------------------------- P1 tetrahedra
def _duffy_integral(X, f):
    """int_T f over the tetrahedron with vertices X (4,3), by the collapsed-cube
    (Duffy) map and 4-point Gauss-Legendre per axis: exact for polynomial f of
    degree <= 4.  Independent of the barycentric-gradient closed forms."""
    g, w = np.polynomial.legendre.leggauss(4)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    tot = 0.0
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            for c, wc in zip(g, w):
                # (a, b, c) in the unit cube -> barycentric (l1, l2, l3)
                l1 = a
                l2 = (1 - a) * b
                l3 = (1 - a) * (1 - b) * c
                jac = (1 - a) ** 2 * (1 - b)
                x = X[0] + l1 * (X[1] - X[0]) + l2 * (X[2] - X[0]) + l3 * (X[3] - X[0])
                tot += wa * wb * wc * jac * f(x)
    return tot * abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)))


def test_p7_tet_element_matrices_by_quadrature():
    """On random tetrahedra: u^T M v = int u v and u^T K v = int grad u . grad v
    for random linear u, v, the integrals taken by Duffy quadrature."""
    rng = np.random.default_rng(17)
    for _ in range(5):
        X = rng.standard_normal((4, 3))
        Ke, Me = fem.tet_matrices(X[None])
        for _ in range(3):
            a, b = rng.standard_normal(3), rng.standard_normal(3)
            a0, b0 = rng.standard_normal(2)
            u, v = X @ a + a0, X @ b + b0           # nodal values of linear functions
            m = _duffy_integral(X, lambda x: (x @ a + a0) * (x @ b + b0))
            k = _duffy_integral(X, lambda x: a @ b)
            assert abs(u @ Me[0] @ v - m) <= 1e-13 * max(1.0, abs(m))
            assert abs(u @ Ke[0] @ v - k) <= 1e-12 * max(1.0, abs(k))
    # a boundary triangle: u^T F v = int u v over the face, by a 2-D collapsed map
    X = rng.standard_normal((3, 3))
    F = fem.tri_mass(X[None])[0]
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    g, w = np.polynomial.legendre.leggauss(4)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    area2 = np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
    ref = sum(wa * wb * (1 - s) * ((X[0] + s * (X[1] - X[0]) + (1 - s) * t * (X[2] - X[0])) @ a)
              * ((X[0] + s * (X[1] - X[0]) + (1 - s) * t * (X[2] - X[0])) @ b)
              for s, wa in zip(g, w) for t, wb in zip(g, w)) * area2
    assert abs((X @ a) @ F @ (X @ b) - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("cells", [(9, 6, 5), (9, 4, 5)])
def test_p7_kuhn_p1_stiffness_is_seven_point_stencil(cells):
    """On the un-jittered Kuhn triangulation of a box of h_x x h_y x h_z cells
    the P1 stiffness of an interior node is the 7-point finite-difference
    stencil scaled by the cell volume (the diagonal couplings of the Kuhn
    tetrahedra cancel), and its mass row sums to the cell volume."""
    nx, ny, nz = cells
    m = W.kuhn_tet_mesh(nx, ny, nz, jitter=0.0, shuffle=False)
    asm = fem.assemble(m)
    K, M = asm["K"].tocsr(), asm["M"].tocsr()
    hx, hy, hz = m["h"]
    V = hx * hy * hz
    for (i, j, k) in ((1, 1, 1), (nx // 2, ny // 2, nz // 2), (nx - 2, ny - 2, nz - 2)):
        r = W.node_id(i, j, k, nx, ny)
        ref = {r: 2 * V * (1 / hx ** 2 + 1 / hy ** 2 + 1 / hz ** 2)}
        for d, hd in zip(((1, 0, 0), (0, 1, 0), (0, 0, 1)), (hx, hy, hz)):
            for sgn in (1, -1):
                ref[W.node_id(i + sgn * d[0], j + sgn * d[1], k + sgn * d[2], nx, ny)] = -V / hd ** 2
        row = K.getrow(r)
        got = {c: v for c, v in zip(row.indices, row.data) if abs(v) > 1e-13 * ref[r]}
        assert set(got) == set(ref)
        for c in ref:
            assert abs(got[c] - ref[c]) <= 1e-13 * ref[r]
        assert abs(M.getrow(r).sum() - V) <= 1e-15


@pytest.mark.parametrize("cells", [(3, 2, 2), (5, 4, 3)])
def test_p7_tet_mesh_invariants(cells):
    """Volume, wall areas, constants in the kernel of K, exact linear patch
    test, bitwise symmetry on the jittered, randomly numbered tet mesh."""
    mesh = W.kuhn_tet_mesh(*cells)
    asm = fem.assemble(mesh)
    K, M = asm["K"], asm["M"]
    n = mesh["n_nodes"]
    Lx, Ly, Lz = W.BOX
    assert abs(M.sum() - Lx * Ly * Lz) <= 1e-13
    areas = [Ly * Lz, Ly * Lz, Lx * Lz, Lx * Lz, Lx * Ly, Lx * Ly]
    for w in range(6):
        assert abs(asm["B0"][w].sum() - areas[w]) <= 1e-13
    assert abs(K - K.T).max() == 0.0 and abs(M - M.T).max() == 0.0
    assert np.abs(K @ np.ones(n)).max() <= 1e-13
    x = mesh["xyz"]
    u = 0.3 * x[:, 0] - 1.2 * x[:, 1] + 0.7 * x[:, 2] + 0.1
    r = K @ u
    inner = np.setdiff1d(np.arange(n), np.unique(mesh["bface"].ravel()))
    assert inner.size > 0
    assert np.abs(r[inner]).max() <= 1e-13 * np.abs(r).max()


def test_p7_tet_plane_wave_second_order():
    """O(h^2) convergence in the L2 (mass) norm to a plane wave with matching
    Robin data on Kuhn tetrahedral meshes refined by halving the cells (the
    coarsest level, k h = 0.7, is still pre-asymptotic: rates rise to 2)."""
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    k = W.wavenumber(200.0)
    beta = np.array([0.5, 0.4 + 0.1j, 0.3, 0.2 - 0.05j, 0.6, 0.45])
    normals = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    errs = []
    for lev in range(3):
        s = 2 ** lev
        mesh = W.kuhn_tet_mesh(9 * s, 6 * s, 5 * s, jitter=0.0)
        S = H.System(mesh, beta)
        pex = np.exp(-1j * k * (mesh["xyz"] @ d))
        f = np.zeros(mesh["n_nodes"], dtype=complex)
        for w in range(6):
            gw = 1j * k * (beta[w] - d @ np.array(normals[w], float)) * pex
            f += S.asm["B0"][w] @ gw
        p = direct.SparseLU(S.operator(k)).solve(f)
        e = p - pex
        errs.append(np.sqrt(np.real(np.vdot(e, S.asm["M"] @ e))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[0] < rates[1] and abs(rates[1] - 2.0) < 0.15, (errs, rates)
