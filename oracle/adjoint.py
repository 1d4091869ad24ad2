"""Receiver sound-pressure energy and its adjoint gradient.

Part of the CPU oracle (test infrastructure only).

Objective: ``J = sum_f sum_r |p_f[r]|^2`` over frequencies f and receiver
nodes r, with ``A(k_f) p_f = f_load`` (operator of the helmholtz module).
For a real parameter theta, ``dJ/dtheta = 2 Re(s^H dp/dtheta)`` with
``s = S p`` (p restricted to the receivers) and
``dp/dtheta = -A^-1 (dA/dtheta) p``, so ``dJ/dtheta = -2 Re(lam^H dA/dtheta p)``
with the adjoint state ``A^H lam = s``.  Because A is complex symmetric,
``A^H = conj(A)`` and ``lam = conj(A^-1 conj(s))``.

With ``dA/deta_e = i k^2 M_e``, ``dA/dRe(beta_w) = i k B0_w`` and
``dA/dIm(beta_w) = -k B0_w``:

    dJ/deta_e     = 2 k^2 Im(lam_e^H M_e p_e)
    dJ/dRe beta_w = 2 k   Im(lam^H B0_w p)
    dJ/dIm beta_w = 2 k   Re(lam^H B0_w p)

summed over frequencies.

With a Dirichlet source (p = g prescribed on the node set D, the system
eliminated to ``A_FF p_F = -A_FD g_D``): ``dp_F/dtheta =
-A_FF^-1 ((dA/dtheta) p)_F`` with the full p (``p_D = g_D``), so the same
formulas hold with the adjoint state of ``A_FF^H lam_F = s_F`` and
``lam_D = 0``; the eliminated full-size system gives that lam_F, its D
entries are set to zero.  The GLS mass coefficient does not depend on beta
or eta, so the formulas are unchanged by it.
"""
from __future__ import annotations

import numpy as np

from . import direct, fem
from .helmholtz import System


def energy(mesh, beta, eta, freqs, g, receivers, c=340.0, system=None, dirichlet=False, gls=False):
    """J and the per-frequency solutions (direct solves)."""
    S = system if system is not None else System(mesh, beta, eta, dirichlet=dirichlet, gls=gls)
    J = 0.0
    ps = []
    for fr in np.atleast_1d(freqs):
        k = 2.0 * np.pi * fr / c
        f_load = S.load(g, k) if S.dirichlet else S.load(g)
        p = direct.SparseLU(S.operator(k)).solve(f_load)
        J += float(np.sum(np.abs(p[receivers]) ** 2))
        ps.append(p)
    return J, ps


def gradient(mesh, beta, eta, freqs, g, receivers, c=340.0, dirichlet=False, gls=False):
    """Returns ``(J, dJ/dbeta (6,2) [Re, Im], dJ/deta (ne,), p list, lam list)``.
    ``eta=None`` is taken as the zero field (its gradient is still returned).
    With ``dirichlet`` the returned lam has its D entries set to zero."""
    hexes = fem.elements(mesh)
    ne = hexes.shape[0]
    eta_v = np.zeros(ne) if eta is None else np.asarray(eta, dtype=np.float64)
    S = System(mesh, beta, eta_v, dirichlet=dirichlet, gls=gls)
    Me = S.asm["Me"]
    J = 0.0
    dbeta = np.zeros((6, 2))
    deta = np.zeros(ne)
    ps, lams = [], []
    for fr in np.atleast_1d(freqs):
        k = 2.0 * np.pi * fr / c
        f_load = S.load(g, k) if S.dirichlet else S.load(g)
        lu = direct.SparseLU(S.operator(k))
        p = lu.solve(f_load)
        J += float(np.sum(np.abs(p[receivers]) ** 2))
        s = np.zeros_like(p)
        s[receivers] = p[receivers]
        lam = np.conj(lu.solve(np.conj(s)))
        lam[S.D] = 0.0
        pe, le = p[hexes], lam[hexes]
        q = np.einsum("eab,eb->ea", Me, pe)
        deta += 2.0 * k * k * np.imag(np.sum(np.conj(le) * q, axis=1))
        for w in range(6):
            val = np.vdot(lam, S.asm["B0"][w] @ p)
            dbeta[w, 0] += 2.0 * k * np.imag(val)
            dbeta[w, 1] += 2.0 * k * np.real(val)
        ps.append(p)
        lams.append(lam)
    return J, dbeta, deta, ps, lams
