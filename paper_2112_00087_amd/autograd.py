"""Receiver sound-pressure energy as a differentiable torch function.

``J = sum_f sum_r |p_f[r]|^2`` with ``A(k_f; beta, eta) p_f = M_patch g``.
The forward pass runs one solve per frequency and the receiver objective
(``hz_receiver_energy``) in the HIP library; the backward pass forms the
adjoint source and runs one adjoint solve per frequency
(``hz_solve_adjoint``) with its gradient kernels, returning dJ/dbeta as
(d/dRe, d/dIm) pairs and dJ/deta per element.  This module only marshals
arguments between torch and the library.
"""
from __future__ import annotations

import numpy as np
import torch


class HelmholtzEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta_ri, eta, model, freqs, g, receivers, opts):
        """beta_ri: (6,2) float64 (Re, Im) per wall; eta: (n_elems,) float64;
        model: a ``Helmholtz``; freqs: Hz; g: nodal patch amplitudes (complex
        device tensor); receivers: node ids (long device tensor); opts: dict of
        solver options."""
        b = beta_ri.detach().cpu().numpy()
        model.set_params(b[:, 0] + 1j * b[:, 1], eta.detach().cpu().numpy())
        f = model.load(g)
        J = 0.0
        ps = []
        for fr in np.atleast_1d(freqs):
            model.set_frequency(fr)
            p, info = model.solve(f, **opts)
            if info["status"] != 0:
                raise RuntimeError(f"forward solve at {fr} Hz did not converge: {info}")
            J += model.receiver_energy(p, receivers)[0]
            ps.append(p)
        ctx.model, ctx.freqs, ctx.receivers, ctx.opts = model, np.atleast_1d(freqs), receivers, opts
        ctx.ps = ps
        return torch.tensor(J, dtype=torch.float64, device=model.device)

    @staticmethod
    def backward(ctx, grad_out):
        model = ctx.model
        deta = torch.zeros(model.ne, dtype=torch.float64, device=model.device)
        dbeta = np.zeros((6, 2))
        for fr, p in zip(ctx.freqs, ctx.ps):
            model.set_frequency(fr)
            _, g = model.receiver_energy(p, ctx.receivers)
            _, db, info = model.solve_adjoint(p, g, dJ_deta=deta, **ctx.opts)
            if info["status"] != 0:
                raise RuntimeError(f"adjoint solve at {fr} Hz did not converge: {info}")
            dbeta += db
        go = grad_out.detach().to(torch.float64)
        gb = torch.as_tensor(dbeta, dtype=torch.float64, device=model.device) * go
        return gb, deta * go, None, None, None, None, None
