"""Seeded synthetic inputs for the box-cavity Helmholtz workloads.

This module is shared by the CPU oracle tests and by the GPU path.  It holds
no finite-element, operator or solver arithmetic: only the node coordinates
and connectivity of a structured box, the tagging of its boundary faces, and
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


def patch_nodes(mesh):
    """Sorted ids of the nodes of the source-patch quads (rim included)."""
    return np.unique(mesh["bface"][mesh["bface_src"] == 1].ravel())


def wavenumber(freq_hz, c=C_SOUND):
    return 2.0 * np.pi * np.asarray(freq_hz, dtype=np.float64) / c


def workload(cfg, elems=None):
    """Seeded inputs for workload ``cfg`` (0..4); ``elems`` overrides the mesh
    size (reduced parity cases) while keeping every other rule.

    Returns a dict: ``mesh``, ``beta`` (6,) complex128, ``g`` (n,) complex128
    nodal patch amplitudes (zero off the patch), ``eta`` (ne,) or None,
    ``receivers`` (r,) int64, ``freqs`` (nf,) Hz, ``parts`` or None.
    """
    spec = CONFIGS[cfg]
    nx, ny, nz = elems if elems is not None else spec["elems"]
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
