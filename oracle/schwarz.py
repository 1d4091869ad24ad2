"""Non-overlapping Schwarz domain decomposition with Robin transmission.

Part of the CPU oracle (test infrastructure only).

Paper Sec. 4 (last part) solves the acoustic problem by a Schwarz method
with absorbing (Robin-type) transmission conditions on the interfaces
between subdomains, optimised in the cited works; the formulae are not in
the paper.  Readings taken here:

* Structured partition of a box mesh into px x py x pz subdomains along
  element planes: the cut of axis d for part a is at element index
  (a * n_d) // p_d.  Interface nodes belong to every subdomain that touches
  them.
* Each subdomain s carries its own Q1 matrices (elements and wall faces it
  owns) plus, on each interface face set G_st shared with a face neighbour
  t, the Robin term T_st = alpha_st M_Gst (M_G: interface-face mass).  The
  default alpha = i k is the absorbing condition for normal incidence in
  the sign convention of the wall admittance (beta = 1).  Two-sided
  conditions (the optimised Schwarz methods of the cited works use a
  different coefficient on each side of an interface): alpha_st = a_lo when
  s is the lower-index side of G_st (its face on the high side of an axis),
  a_hi when it is the higher-index side.
* Local problem: (A~_s + sum_t T_st) u_s = f_s + sum_t R_st^T lam_st, with
  f_s = (R_s f) / multiplicity, so that sum_s R_s^T f_s = f.
* Transmission: lam_st <- (T_st + T_ts) R_ts u_t - lam_ts, with
  T_st + T_ts = (a_lo + a_hi) M_Gst.  At the fixed point u_s = u_t on G_st
  and the assembled equations hold on interface nodes, so the glued
  solution equals the global one for any coefficients.
* One multiplier vector per ordered pair of face neighbours, on all nodes
  of G_st (edges and corners included), which handles cross points.
* Glue: average of the duplicated interface values.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import direct, fem
from .helmholtz import System


def cuts(n, p):
    return [(a * n) // p for a in range(p + 1)]


def partition(mesh, parts):
    """List of subdomains: element ranges ((x0,x1),(y0,y1),(z0,z1)) with the
    subdomain id s = a + px (b + py c)."""
    nx, ny, nz = mesh["elems"]
    px, py, pz = parts
    cx, cy, cz = cuts(nx, px), cuts(ny, py), cuts(nz, pz)
    subs = []
    for c in range(pz):
        for b in range(py):
            for a in range(px):
                subs.append(((cx[a], cx[a + 1]), (cy[b], cy[b + 1]), (cz[c], cz[c + 1])))
    return subs


def _gid(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def local_mesh(mesh, parts, s):
    """Mesh of subdomain s with local node numbering; boundary faces carry
    wall tags 0..5 (global walls) or 6 + 2 d + side (interface towards the
    neighbour across the low (side 0) or high (side 1) face of axis d)."""
    nx, ny, nz = mesh["elems"]
    subs = partition(mesh, parts)
    rng = subs[s]
    lo = [r[0] for r in rng]
    ln = [r[1] - r[0] for r in rng]
    I, J, K = np.meshgrid(np.arange(ln[0] + 1), np.arange(ln[1] + 1), np.arange(ln[2] + 1), indexing="ij")
    I, J, K = (A.transpose(2, 1, 0).ravel() for A in (I, J, K))
    l2g = _gid(I + lo[0], J + lo[1], K + lo[2], nx, ny)
    xyz = mesh["xyz"][l2g]
    ei, ej, ek = np.meshgrid(np.arange(ln[0]), np.arange(ln[1]), np.arange(ln[2]), indexing="ij")
    ei, ej, ek = (A.transpose(2, 1, 0).ravel() for A in (ei, ej, ek))
    hexes = np.empty((ei.size, 8), dtype=np.int64)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                hexes[:, a + 2 * b + 4 * c] = _gid(ei + a, ej + b, ek + c, ln[0], ln[1])
    g2l = -np.ones(mesh["xyz"].shape[0], dtype=np.int64)
    g2l[l2g] = np.arange(l2g.size)
    # global wall faces owned by this subdomain (owner = subdomain of the adjacent element)
    bf = mesh["bface"].astype(np.int64)
    gi = bf % (nx + 1)
    gj = (bf // (nx + 1)) % (ny + 1)
    gk = bf // ((nx + 1) * (ny + 1))
    e_i = np.minimum(gi.min(1), nx - 1)
    e_j = np.minimum(gj.min(1), ny - 1)
    e_k = np.minimum(gk.min(1), nz - 1)
    own = ((e_i >= rng[0][0]) & (e_i < rng[0][1]) & (e_j >= rng[1][0]) & (e_j < rng[1][1])
           & (e_k >= rng[2][0]) & (e_k < rng[2][1]))
    faces = [g2l[bf[own]]]
    tags = [mesh["bface_tag"][own]]
    src = [mesh["bface_src"][own]]
    # interface faces
    counts = (nx, ny, nz)
    for d in range(3):
        a1, a2 = [q for q in range(3) if q != d]
        for side in range(2):
            plane = rng[d][side]
            if plane in (0, counts[d]):
                continue
            u, v = np.meshgrid(np.arange(ln[a1]), np.arange(ln[a2]), indexing="ij")
            u, v = u.T.ravel(), v.T.ravel()
            q = np.empty((u.size, 4), dtype=np.int64)
            for bb in range(2):
                for aa in range(2):
                    idx = [None, None, None]
                    idx[d] = np.full(u.size, side * ln[d])
                    idx[a1] = u + aa
                    idx[a2] = v + bb
                    q[:, aa + 2 * bb] = _gid(idx[0], idx[1], idx[2], ln[0], ln[1])
            faces.append(q)
            tags.append(np.full(u.size, 6 + 2 * d + side, dtype=np.int32))
            src.append(np.zeros(u.size, dtype=np.uint8))
    return dict(xyz=xyz, hex=hexes, bface=np.concatenate(faces), bface_tag=np.concatenate(tags),
                bface_src=np.concatenate(src), l2g=l2g, elems=tuple(ln), n_nodes=l2g.size,
                n_elems=hexes.shape[0], range=rng)


def neighbours(parts):
    """Ordered face-neighbour pairs (s, t, d, side): t is across the
    low (side 0) or high (side 1) face of axis d of s."""
    px, py, pz = parts
    out = []
    for c in range(pz):
        for b in range(py):
            for a in range(px):
                s = a + px * (b + py * c)
                pos = [a, b, c]
                for d in range(3):
                    for side in range(2):
                        q = list(pos)
                        q[d] += 1 if side else -1
                        if 0 <= q[d] < parts[d]:
                            out.append((s, q[0] + px * (q[1] + py * q[2]), d, side))
    return out


class Schwarz:
    """Subdomain operators, interface maps and the Schwarz iteration."""

    def __init__(self, mesh, parts, beta, eta, k, f, alpha=None):
        """alpha: one coefficient for both sides (default i k), or a pair
        (a_lo, a_hi) of two-sided coefficients."""
        self.mesh, self.parts, self.k = mesh, parts, k
        if alpha is None:
            alpha = 1j * k
        if np.ndim(alpha) == 0:
            self.a_lo = self.a_hi = complex(alpha)
        else:
            self.a_lo, self.a_hi = complex(alpha[0]), complex(alpha[1])
        self.subs = partition(mesh, parts)
        self.ns = len(self.subs)
        n = mesh["xyz"].shape[0]
        self.loc = [local_mesh(mesh, parts, s) for s in range(self.ns)]
        mult = np.zeros(n)
        for L in self.loc:
            mult[L["l2g"]] += 1
        self.mult = mult
        self.A, self.lu, self.f = [], [], []
        self.MG = {}
        for s, L in enumerate(self.loc):
            asm = fem.assemble(dict(L, bface_tag=np.where(L["bface_tag"] < 6, L["bface_tag"], 0),
                                    bface_src=L["bface_src"]), with_element_mass=eta is not None)
            K, M = asm["K"], asm["M"]
            A = K.astype(complex) - (k * k) * M
            if eta is not None:
                eloc = np.asarray(eta)[self._global_elements(L)]
                A = A + (1j * k * k) * fem.element_weighted_mass(L, asm["Me"], eloc)
            bf = L["bface"].astype(np.int64)
            Fe = fem.quad_mass(L["xyz"][bf])
            nl = L["n_nodes"]
            for w in range(6):
                sel = L["bface_tag"] == w
                if np.any(sel) and beta[w] != 0:
                    A = A + (1j * k * beta[w]) * fem.Pattern(bf[sel], nl).matrix(Fe[sel])
            for tag in range(6, 12):
                sel = L["bface_tag"] == tag
                if np.any(sel):
                    MG = fem.Pattern(bf[sel], nl).matrix(Fe[sel])
                    self.MG[(s, tag)] = MG
                    # tag 6 + 2d + side: side 1 is the high face (s the lower-index side)
                    A = A + (self.a_lo if (tag - 6) % 2 == 1 else self.a_hi) * MG
            A = sp.csr_matrix(A)
            self.A.append(A)
            self.lu.append(direct.SparseLU(A))
            self.f.append(np.asarray(f)[L["l2g"]] / mult[L["l2g"]])
        # interface pairs: nodes of G_st in s and in t
        self.pairs = []
        for (s, t, d, side) in neighbours(parts):
            tag = 6 + 2 * d + side
            Ls, Lt = self.loc[s], self.loc[t]
            sel = Ls["bface_tag"] == tag
            gnodes = np.unique(Ls["l2g"][Ls["bface"][sel].ravel()])
            g2s = {g: i for i, g in enumerate(Ls["l2g"])}
            g2t = {g: i for i, g in enumerate(Lt["l2g"])}
            ins = np.array([g2s[g] for g in gnodes])
            int_ = np.array([g2t[g] for g in gnodes])
            MG = self.MG[(s, tag)][ins][:, ins]
            self.pairs.append(dict(s=s, t=t, tag=tag, g=gnodes, ins=ins, int=int_, MG=sp.csr_matrix(MG)))
        self.index = {(p["s"], p["t"]): i for i, p in enumerate(self.pairs)}

    def _global_elements(self, L):
        nx, ny, nz = self.mesh["elems"]
        (x0, x1), (y0, y1), (z0, z1) = L["range"]
        ei, ej, ek = np.meshgrid(np.arange(x0, x1), np.arange(y0, y1), np.arange(z0, z1), indexing="ij")
        ei, ej, ek = (A.transpose(2, 1, 0).ravel() for A in (ei, ej, ek))
        return ei + nx * (ej + ny * ek)

    def local_solve(self, lams, with_f=True):
        us = []
        for s in range(self.ns):
            rhs = self.f[s].astype(complex) if with_f else np.zeros(self.loc[s]["n_nodes"], complex)
            rhs = rhs.copy()
            for i, p in enumerate(self.pairs):
                if p["s"] == s:
                    np.add.at(rhs, p["ins"], lams[i])
            us.append(self.lu[s].solve(rhs))
        return us

    def update(self, lams, us):
        """lam_st <- (a_lo + a_hi) M_G R_ts u_t - lam_ts."""
        new = []
        for i, p in enumerate(self.pairs):
            j = self.index[(p["t"], p["s"])]
            # lam_ts is indexed by the same global nodes, in t's order of G_ts == G_st
            lam_ts = lams[j][np.searchsorted(self.pairs[j]["g"], p["g"])]
            new.append((self.a_lo + self.a_hi) * (p["MG"] @ us[p["t"]][p["int"]]) - lam_ts)
        return new

    def glue(self, us):
        n = self.mesh["xyz"].shape[0]
        acc = np.zeros(n, complex)
        for s, u in enumerate(us):
            np.add.at(acc, self.loc[s]["l2g"], u)
        return acc / self.mult

    def zero_lams(self):
        return [np.zeros(p["g"].size, complex) for p in self.pairs]

    def richardson(self, iters, A_global=None, f_global=None):
        """Plain Schwarz iteration from lam = 0.  Returns (u, lams, history)
        with history rows (||lam_new - lam||, global relres of the glued u)."""
        lams = self.zero_lams()
        hist = []
        u = None
        for _ in range(iters):
            us = self.local_solve(lams)
            new = self.update(lams, us)
            dl = np.sqrt(sum(np.linalg.norm(a - b) ** 2 for a, b in zip(new, lams)))
            u = self.glue(us)
            rel = (np.linalg.norm(f_global - A_global @ u) / np.linalg.norm(f_global)
                   if A_global is not None else np.nan)
            hist.append((dl, rel))
            lams = new
        return u, lams, np.array(hist)

    def interface_operator(self):
        """(I - B) as a scipy LinearOperator on the stacked multipliers, and c."""
        import scipy.sparse.linalg as spla
        sizes = [p["g"].size for p in self.pairs]
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        N = int(off[-1])

        def split(v):
            return [v[off[i]:off[i + 1]] for i in range(len(sizes))]

        def mv(v):
            L = split(np.asarray(v, dtype=complex).ravel())
            return v.ravel() - np.concatenate(self.update(L, self.local_solve(L, with_f=False)))

        c = np.concatenate(self.update(self.zero_lams(), self.local_solve(self.zero_lams(), True)))
        return spla.LinearOperator((N, N), matvec=mv, dtype=complex), c, split

    def interface_matrix(self):
        """Dense (I - B) and c of the interface system (I - B) lam = c (tiny cases)."""
        sizes = [p["g"].size for p in self.pairs]
        off = np.concatenate([[0], np.cumsum(sizes)])
        N = off[-1]

        def split(v):
            return [v[off[i]:off[i + 1]] for i in range(len(sizes))]

        c = np.concatenate(self.update(self.zero_lams(), self.local_solve(self.zero_lams(), True)))
        cols = []
        for j in range(N):
            e = np.zeros(N, complex)
            e[j] = 1.0
            L = split(e)
            B = np.concatenate(self.update(L, self.local_solve(L, with_f=False)))
            cols.append(e - B)
        return np.stack(cols, axis=1), c, split
