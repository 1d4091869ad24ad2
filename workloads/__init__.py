"""Seeded synthetic inputs for the box-cavity Helmholtz workloads.

This module is shared by the CPU oracle tests and by the GPU path.  It holds
no finite-element, operator or solver arithmetic: only the node coordinates
and connectivity of a structured box (or of an unstructured hexahedral mesh
of the same box), the tagging of its boundary faces, and
the seeded random draws (wall admittances, roof-patch forcing amplitudes,
absorption field, receiver nodes) that stand in for the paper's car
compartment and sun-roof data (paper Sec. 3.2, Helmholtz equation and the
sun-roof boundary data that follows it).

Conventions
-----------
* Node id ``i + (nx+1)*(j + (ny+1)*k)`` (x fastest), coordinates
  ``(i*hx, j*hy, k*hz)``.
* Element id ``ei + nx*(ej + ny*ek)``; its 8 nodes are listed in tensor
  order: local node ``a + 2*b + 4*c`` sits at ``(ei+a, ej+b, ek+c)``.
* Walls are numbered 0..5 = x-, x+, y-, y+, z- (floor), z+ (roof).  A wall
  quad lists its 4 nodes in tensor order over the two in-plane axes (the
  lower-numbered axis fastest).
* A roof quad belongs to the sun-roof source patch iff its centroid lies in
  ``[0.6, 1.2] x [0.3, 0.9]`` (a 0.6 m x 0.6 m opening centred on the roof).
* Workloads 5 and 6 are unstructured (:func:`kuhn_hex_mesh`,
  :func:`kuhn_tet_mesh`; generators seeded ``SEED + 1000 + cfg``); their node
  ids follow no spatial order.  Workload 6 holds tetrahedra (key ``tet``,
  triangles in ``bface``).
* Draw order for one workload, from ``numpy.random.default_rng(SEED + cfg)``:
  (1) wall admittances, per wall Re then Im (seeded-wall workloads only);
  (2) patch amplitudes, all Re then all Im, in ascending node id;
  (3) the per-element absorption field; (4) the receiver nodes.
"""
from __future__ import annotations

import numpy as np

SEED = 211200087
BOX = (1.8, 1.2, 1.0)          # cavity lengths (m)
C_SOUND = 340.0                # speed of sound (m/s)
RHO = 1.2                      # density (kg/m^3), carried but unused by the operator
PATCH = ((0.6, 1.2), (0.3, 0.9))
WALLS = ("x-", "x+", "y-", "y+", "z-", "z+")
FLOOR_BETA = 0.01 + 0.002j

# name, elements per axis, frequencies (Hz), wall rule, absorption, receivers
CONFIGS = {
    0: dict(name="cavity-20x12x10-100Hz", elems=(20, 12, 10), freqs=(100.0,),
            walls="floor", eta=False, receivers=0),
    1: dict(name="cavity-160x96x80-250Hz", elems=(160, 96, 80), freqs=(250.0,),
            walls="seeded", eta=False, receivers=0),
    2: dict(name="sweep-80x48x40-64f-20-300Hz", elems=(80, 48, 40),
            freqs=tuple(np.linspace(20.0, 300.0, 64)), walls="floor", eta=False,
            receivers=0),
    3: dict(name="schwarz-200x120x100-24sub-150Hz", elems=(200, 120, 100),
            freqs=(150.0,), walls="seeded", eta=False, receivers=0,
            parts=(4, 3, 2)),
    4: dict(name="adjoint-80x48x40-16f-50-200Hz", elems=(80, 48, 40),
            freqs=tuple(np.linspace(50.0, 200.0, 16)), walls="seeded", eta=True,
            receivers=16),
    # unstructured: elems are the Kuhn cells (24 hexahedra each), nodes randomly numbered
    5: dict(name="kuhn-48x32x32-250Hz", elems=(48, 32, 32), freqs=(250.0,),
            walls="seeded", eta=False, receivers=0, mesh="kuhn"),
    # unstructured tetrahedra: the Kuhn tetrahedra of the cells themselves (P1)
    6: dict(name="kuhn-tet-144x96x96-250Hz", elems=(144, 96, 96), freqs=(250.0,),
            walls="seeded", eta=False, receivers=0, mesh="kuhn-tet"),
}


def node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def box_mesh(nx, ny, nz, lengths=BOX, patch=PATCH):
    """Structured hexahedral mesh of the box ``[0,Lx]x[0,Ly]x[0,Lz]``.

    Returns a dict with ``xyz`` (n,3) float64, ``hex`` (ne,8) int32,
    ``bface`` (nb,4) int32, ``bface_tag`` (nb,) int32, ``bface_src`` (nb,)
    uint8, plus the element counts and spacings.
    """
    Lx, Ly, Lz = lengths
    hx, hy, hz = Lx / nx, Ly / ny, Lz / nz
    I, J, K = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                          indexing="ij")
    # flatten in node-id order (x fastest)
    I = I.transpose(2, 1, 0).ravel()
    J = J.transpose(2, 1, 0).ravel()
    K = K.transpose(2, 1, 0).ravel()
    xyz = np.stack([I * hx, J * hy, K * hz], axis=1).astype(np.float64)

    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ei = ei.transpose(2, 1, 0).ravel()
    ej = ej.transpose(2, 1, 0).ravel()
    ek = ek.transpose(2, 1, 0).ravel()
    hexes = np.empty((ei.size, 8), dtype=np.int64)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                hexes[:, a + 2 * b + 4 * c] = node_id(ei + a, ej + b, ek + c, nx, ny)

    faces, tags, src = [], [], []
    counts = (nx, ny, nz)
    for axis in range(3):
        ax1, ax2 = [d for d in range(3) if d != axis]
        u, v = np.meshgrid(np.arange(counts[ax1]), np.arange(counts[ax2]), indexing="ij")
        u = u.T.ravel()
        v = v.T.ravel()
        for side in range(2):
            q = np.empty((u.size, 4), dtype=np.int64)
            for bb in range(2):
                for aa in range(2):
                    idx = [None, None, None]
                    idx[axis] = np.full(u.size, side * counts[axis])
                    idx[ax1] = u + aa
                    idx[ax2] = v + bb
                    q[:, aa + 2 * bb] = node_id(idx[0], idx[1], idx[2], nx, ny)
            faces.append(q)
            tags.append(np.full(u.size, 2 * axis + side, dtype=np.int32))
            if axis == 2 and side == 1:
                cx = (u + 0.5) * hx
                cy = (v + 0.5) * hy
                inside = ((cx >= patch[0][0]) & (cx <= patch[0][1]) &
                          (cy >= patch[1][0]) & (cy <= patch[1][1]))
                src.append(inside.astype(np.uint8))
            else:
                src.append(np.zeros(u.size, dtype=np.uint8))
    return dict(
        xyz=xyz,
        hex=hexes.astype(np.int32),
        bface=np.concatenate(faces).astype(np.int32),
        bface_tag=np.concatenate(tags),
        bface_src=np.concatenate(src),
        elems=(nx, ny, nz), h=(hx, hy, hz), lengths=tuple(lengths),
        n_nodes=xyz.shape[0], n_elems=hexes.shape[0],
    )


# local vertex pairs of a tetrahedron's edges, in this order
_TET_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _kuhn_tets(nx, ny, nz, lengths, jitter, rng):
    """Jittered grid vertices and the positively oriented Kuhn tetrahedra of
    its cells (6 per cell around the main diagonal, conforming)."""
    Lx, Ly, Lz = lengths
    h = np.array([Lx / nx, Ly / ny, Lz / nz])
    nv = (nx + 1) * (ny + 1) * (nz + 1)
    vid = np.arange(nv)
    gi = np.stack([vid % (nx + 1), (vid // (nx + 1)) % (ny + 1), vid // ((nx + 1) * (ny + 1))], 1)
    top = np.array([nx, ny, nz])
    free = (gi > 0) & (gi < top)
    vx = gi * h + np.where(free, rng.uniform(-jitter, jitter, size=(nv, 3)), 0.0) * h
    # cells -> 6 Kuhn tetrahedra: corner bits x=1, y=2, z=4; path 0 -> 7
    ci, cj, ck = [a.ravel() for a in np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")]
    corner = np.stack([node_id(ci + (b & 1), cj + ((b >> 1) & 1), ck + ((b >> 2) & 1), nx, ny)
                       for b in range(8)], 1)
    tets = []
    for p0, p1, _ in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        b1 = 1 << p0
        b2 = b1 | (1 << p1)
        tets.append(np.stack([corner[:, 0], corner[:, b1], corner[:, b2], corner[:, 7]], 1))
    tet = np.concatenate(tets)
    d = vx[tet[:, 1:]] - vx[tet[:, :1]]
    vol = np.einsum("ij,ij->i", d[:, 0], np.cross(d[:, 1], d[:, 2]))
    neg = vol < 0
    tet[neg, 2], tet[neg, 3] = tet[neg, 3].copy(), tet[neg, 2].copy()
    if not np.all(np.abs(vol) > 1e-3 * h.prod()):
        raise ValueError("jitter too large: a tetrahedron degenerates")
    return vx, gi, top, tet, h


def _wall_tags(gi, top, tri):
    """Wall id of boundary triangles given by their grid-vertex ids."""
    g3 = gi[tri]
    tag = np.full(tri.shape[0], -1)
    for ax in range(3):
        tag = np.where(np.all(g3[:, :, ax] == 0, 1), 2 * ax, tag)
        tag = np.where(np.all(g3[:, :, ax] == top[ax], 1), 2 * ax + 1, tag)
    assert np.all(tag >= 0)
    return tag.astype(np.int32)


def _faces_once(tet, nv):
    """(tetrahedron, opposite local vertex) of the faces used by one
    tetrahedron only (the boundary), plus per-tetrahedron face keys."""
    fkey = np.stack([np.sort(np.delete(tet, o, axis=1), 1) for o in range(4)], 1)  # face opposite o
    fkey = (fkey[..., 0].astype(np.int64) * nv + fkey[..., 1]) * nv + fkey[..., 2]
    uf, finv, fcnt = np.unique(fkey.ravel(), return_inverse=True, return_counts=True)
    once = np.nonzero(fcnt[finv] == 1)[0]
    return once // 4, once % 4, uf, finv.reshape(tet.shape[0], 4)


def _patch_flags(btag, cen, patch):
    return ((btag == 5) & (cen[:, 0] >= patch[0][0]) & (cen[:, 0] <= patch[0][1]) &
            (cen[:, 1] >= patch[1][0]) & (cen[:, 1] <= patch[1][1])).astype(np.uint8)


def kuhn_tet_mesh(nx, ny, nz, lengths=BOX, patch=PATCH, jitter=0.1, seed=SEED, shuffle=True):
    """Unstructured tetrahedral mesh of the box: the jittered Kuhn
    tetrahedra of ``nx x ny x nz`` cells (see :func:`kuhn_hex_mesh`),
    boundary triangles tagged by wall, nodes, elements and faces in a seeded
    random order with ``shuffle``.  Returns ``xyz``, ``tet`` (ne,4) int32,
    ``bface`` (nb,3) triangles and the tags of :func:`box_mesh`."""
    rng = np.random.default_rng(seed)
    vx, gi, top, tet, h = _kuhn_tets(nx, ny, nz, lengths, jitter, rng)
    nv = vx.shape[0]
    bt, bo, _, _ = _faces_once(tet, nv)
    tri = np.stack([tet[bt, v] for v in range(4)], 1)
    keep = np.arange(4)[None, :] != bo[:, None]
    tri = tri[keep].reshape(-1, 3)
    btag = _wall_tags(gi, top, tri)
    src = _patch_flags(btag, vx[tri].mean(1), patch)
    xyz = vx
    if shuffle:
        pn = rng.permutation(nv)
        inv = np.empty(nv, dtype=np.int64)
        inv[pn] = np.arange(nv)
        xyz = vx[inv]
        tet = pn[tet][rng.permutation(tet.shape[0])]
        fo = rng.permutation(tri.shape[0])
        tri, btag, src = pn[tri][fo], btag[fo], src[fo]
    return dict(
        xyz=np.ascontiguousarray(xyz), tet=tet.astype(np.int32), bface=tri.astype(np.int32),
        bface_tag=btag, bface_src=src, elems=(0, 0, 0), cells=(nx, ny, nz), h=tuple(h),
        lengths=tuple(lengths), n_nodes=nv, n_elems=tet.shape[0],
    )


def kuhn_hex_mesh(nx, ny, nz, lengths=BOX, patch=PATCH, jitter=0.1, seed=SEED, shuffle=True):
    """Unstructured all-hexahedral mesh of the box (stand-in for the paper's
    unstructured compartment mesh, Sec. 3.2).

    The box is cut into ``nx x ny x nz`` cells, each cell into the 6 Kuhn
    tetrahedra that share its main diagonal (conforming across cells), and
    each tetrahedron into 4 hexahedra, one per corner, whose nodes are the
    corner, the 3 edge midpoints, the 3 face centroids and the centroid next
    to it (all faces planar).  Node valences then range from 4 to 24
    elements, so matrix rows range from 12 to 75 entries.

    Grid vertices move by ``uniform(-jitter, jitter)`` cell widths along
    every axis on which they are not on a wall (walls stay planar).  With
    ``shuffle`` the nodes, elements and boundary faces are numbered in a
    seeded random order, as an unstructured mesh generator may leave them.

    Returns the same keys as :func:`box_mesh` (``elems`` is the cell grid;
    the mesh is not a structured box).
    """
    rng = np.random.default_rng(seed)
    vx, gi, top, tet, h = _kuhn_tets(nx, ny, nz, lengths, jitter, rng)
    nv = vx.shape[0]
    nt = tet.shape[0]

    # global ids of edge midpoints, face centroids and cell centroids
    ekey = np.stack([np.sort(tet[:, list(e)], 1) for e in _TET_EDGES], 1)          # (nt,6,2)
    ekey = ekey[..., 0].astype(np.int64) * nv + ekey[..., 1]
    ue, einv = np.unique(ekey.ravel(), return_inverse=True)
    eid = nv + einv.reshape(nt, 6)
    bt, bo, uf, finv = _faces_once(tet, nv)
    fid = nv + ue.size + finv
    gid = nv + ue.size + uf.size + np.arange(nt)
    n = nv + ue.size + uf.size + nt
    xyz = np.empty((n, 3))
    xyz[:nv] = vx
    xyz[nv:nv + ue.size] = 0.5 * (vx[ue // nv] + vx[ue % nv])
    fa, fb, fc = uf // (nv * nv), (uf // nv) % nv, uf % nv
    xyz[nv + ue.size:nv + ue.size + uf.size] = (vx[fa] + vx[fb] + vx[fc]) / 3.0
    xyz[nv + ue.size + uf.size:] = vx[tet].mean(1)

    def mid(i, j):
        return eid[:, _TET_EDGES.index((min(i, j), max(i, j)))]

    def face(*v):
        return fid[:, ({0, 1, 2, 3} - set(v)).pop()]

    hexes = []
    for i in range(4):
        j, k, l = [v for v in range(4) if v != i]
        if i % 2:
            j, k = k, j          # keep the corner's axis triple right-handed
        hexes.append(np.stack([tet[:, i], mid(i, j), mid(i, k), face(i, j, k),
                               mid(i, l), face(i, j, l), face(i, k, l), gid], 1))
    hexes = np.concatenate(hexes)
    X = xyz[hexes]
    jac = np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 4] - X[:, 0]))
    assert np.all(jac > 0), "hexahedron orientation"

    # boundary: tetrahedron faces used once; 3 quads per triangle
    tri = np.array([[v for v in range(4) if v != o] for o in range(4)])[bo]   # local ids, ascending
    eidx = np.full((4, 4), -1)
    for q, (x, y) in enumerate(_TET_EDGES):
        eidx[x, y] = eidx[y, x] = q
    tag = _wall_tags(gi, top, tet[bt[:, None], tri])
    quads, tags = [], []
    for c in range(3):
        a_, b_, c_ = tri[:, c], tri[:, (c + 1) % 3], tri[:, (c + 2) % 3]
        quads.append(np.stack([tet[bt, a_], eid[bt, eidx[a_, b_]], eid[bt, eidx[a_, c_]], fid[bt, bo]], 1))
        tags.append(tag)
    bface = np.concatenate(quads)
    btag = np.concatenate(tags).astype(np.int32)
    src = _patch_flags(btag, xyz[bface].mean(1), patch)

    if shuffle:
        pn = rng.permutation(n)           # old id -> new id
        inv = np.empty(n, dtype=np.int64)
        inv[pn] = np.arange(n)
        xyz = xyz[inv]
        hexes = pn[hexes][rng.permutation(hexes.shape[0])]
        fo = rng.permutation(bface.shape[0])
        bface, btag, src = pn[bface][fo], btag[fo], src[fo]
    return dict(
        xyz=np.ascontiguousarray(xyz), hex=hexes.astype(np.int32), bface=bface.astype(np.int32),
        bface_tag=btag, bface_src=src, elems=(0, 0, 0), cells=(nx, ny, nz), h=tuple(h / 2.0),
        lengths=tuple(lengths), n_nodes=n, n_elems=hexes.shape[0],
    )


def patch_nodes(mesh):
    """Sorted ids of the nodes of the source-patch quads (rim included)."""
    return np.unique(mesh["bface"][mesh["bface_src"] == 1].ravel())


def wavenumber(freq_hz, c=C_SOUND):
    return 2.0 * np.pi * np.asarray(freq_hz, dtype=np.float64) / c


def workload(cfg, elems=None):
    """Seeded inputs for workload ``cfg`` (0..6); ``elems`` overrides the mesh
    size (reduced parity cases) while keeping every other rule.

    Returns a dict: ``mesh``, ``beta`` (6,) complex128, ``g`` (n,) complex128
    nodal patch amplitudes (zero off the patch), ``eta`` (ne,) or None,
    ``receivers`` (r,) int64, ``freqs`` (nf,) Hz, ``parts`` or None.
    """
    spec = CONFIGS[cfg]
    nx, ny, nz = elems if elems is not None else spec["elems"]
    if spec.get("mesh") == "kuhn":
        mesh = kuhn_hex_mesh(nx, ny, nz, seed=SEED + 1000 + cfg)
    elif spec.get("mesh") == "kuhn-tet":
        mesh = kuhn_tet_mesh(nx, ny, nz, seed=SEED + 1000 + cfg)
    else:
        mesh = box_mesh(nx, ny, nz)
    rng = np.random.default_rng(SEED + cfg)
    beta = np.zeros(6, dtype=np.complex128)
    if spec["walls"] == "floor":
        beta[4] = FLOOR_BETA
    else:
        for w in range(6):
            re = rng.uniform(0.0, 0.05)
            im = rng.uniform(-0.01, 0.01)
            beta[w] = re + 1j * im
    pn = patch_nodes(mesh)
    g = np.zeros(mesh["n_nodes"], dtype=np.complex128)
    gre = rng.standard_normal(pn.size)
    gim = rng.standard_normal(pn.size)
    g[pn] = gre + 1j * gim
    eta = rng.uniform(0.0, 0.02, size=mesh["n_elems"]) if spec["eta"] else None
    receivers = np.zeros(0, dtype=np.int64)
    if spec["receivers"]:
        i = np.arange(1, nx)
        j = np.arange(1, ny)
        k = np.arange(1, nz)
        I, J, K = np.meshgrid(i, j, k, indexing="ij")
        interior = np.sort(node_id(I.ravel(), J.ravel(), K.ravel(), nx, ny))
        receivers = rng.choice(interior, size=min(spec["receivers"], interior.size),
                               replace=False).astype(np.int64)
    return dict(cfg=cfg, name=spec["name"], mesh=mesh, beta=beta, g=g, eta=eta,
                receivers=receivers, freqs=np.asarray(spec["freqs"], dtype=np.float64),
                parts=spec.get("parts"), c=C_SOUND, rho=RHO)
