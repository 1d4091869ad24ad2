"""Right-Jacobi preconditioned Krylov solvers in complex128.

Part of the CPU oracle (test infrastructure only).

Paper Sec. 4 solves the acoustic system with preconditioned Krylov methods
(P-BiCGSTAB among them) in complex double precision; the preconditioner
type is not stated.  Readings taken here:

* Preconditioner: Jacobi, ``D = diag(A)`` (complex), applied on the right,
  so the iteration runs on ``A D^-1 u = f`` with ``x = D^-1 u`` and the
  residual it tracks is the true residual ``f - A x``.
* Stop when the true relative residual ``||f - A x|| / ||f||`` reaches
  ``tol``; it is recomputed before returning.
* Inner products ``<a, b> = a^H b``.

GMRES(m) is restarted GMRES with modified Gram-Schmidt Arnoldi and complex
Givens rotations: for a column pair (a, b), ``rho = sqrt(|a|^2 + |b|^2)``,
``c = |a| / rho``, ``s = (a/|a|) conj(b) / rho`` (``c = 0, s = 1`` when
``a = 0``), which maps (a, b) to (a/|a| rho, 0).  A happy breakdown
(zero subdiagonal) ends the cycle.

BiCGStab is van der Vorst's stabilised bi-conjugate gradient method with
shadow residual ``r^ = r0``, an early exit when ``||s||`` is small, and a
restart with ``r^ = r`` when ``rho`` or ``omega`` breaks down.
"""
from __future__ import annotations

import numpy as np


class Result:
    def __init__(self, x, status, iters, matvecs, relres, history):
        self.x, self.status, self.iters, self.matvecs = x, status, iters, matvecs
        self.relres, self.history = relres, history

    def __repr__(self):
        return (f"Result(status={self.status}, iters={self.iters}, "
                f"matvecs={self.matvecs}, relres={self.relres:.3e})")


def _dinv(A, precond):
    n = A.shape[0]
    if precond == "jacobi":
        return 1.0 / A.diagonal().astype(np.complex128)
    return np.ones(n, dtype=np.complex128)


def givens(a, b):
    """Complex Givens pair (c real, s complex) zeroing b against a."""
    rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    if rho == 0.0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    return abs(a) / rho, (a / abs(a)) * np.conj(b) / rho


def gmres(A, f, m=30, tol=1e-8, max_matvec=20000, x0=None, precond="jacobi",
          record_cycles=False):
    f = np.asarray(f, dtype=np.complex128)
    n = f.size
    dinv = _dinv(A, precond)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nf = np.linalg.norm(f)
    matvecs, iters, hist, cycles = 0, 0, [], []
    if nf == 0.0:
        return Result(np.zeros(n, dtype=np.complex128), 0, 0, 0, 0.0, hist)
    status = 1
    while True:
        r = f - A @ x
        matvecs += 1
        beta = np.linalg.norm(r)
        hist.append(beta / nf)
        if beta / nf <= tol:
            status = 0
            break
        if matvecs >= max_matvec:
            break
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        cyc = []
        for j in range(m):
            w = A @ (dinv * V[j])
            matvecs += 1
            iters += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            for i in range(j):
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * b
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            cyc.append(abs(g[j + 1]) / nf)
            if hnext == 0.0 or abs(g[j + 1]) / nf <= tol or matvecs >= max_matvec:
                break
            V[j + 1] = w / hnext
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + dinv * (V[:k].T @ y)
        cycles.append(cyc)
    res = Result(x, status, iters, matvecs, np.linalg.norm(f - A @ x) / nf, hist)
    if record_cycles:
        res.cycles = cycles
    return res


def bicgstab(A, f, tol=1e-8, max_matvec=20000, x0=None, precond="jacobi",
             max_iters=None):
    f = np.asarray(f, dtype=np.complex128)
    n = f.size
    dinv = _dinv(A, precond)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return Result(np.zeros(n, dtype=np.complex128), 0, 0, 0, 0.0, [])
    matvecs, iters, hist, status = 0, 0, [], 1
    while status != 0:
        # (re)start from the true residual of the current iterate
        r = f - A @ x
        matvecs += 1
        hist.append(np.linalg.norm(r) / nf)
        if hist[-1] <= tol:
            status = 0
            break
        rhat = r.copy()
        rho_old = alpha = omega = 1.0 + 0.0j
        v = np.zeros(n, dtype=np.complex128)
        p = np.zeros(n, dtype=np.complex128)
        done = False
        while matvecs + 2 <= max_matvec:
            if max_iters is not None and iters >= max_iters:
                break
            rho = np.vdot(rhat, r)
            if abs(rho) < 1e-300 * np.linalg.norm(rhat) * np.linalg.norm(r) or omega == 0:
                rhat = r.copy()
                rho = np.vdot(rhat, r)
                rho_old = alpha = omega = 1.0 + 0.0j
                v[:] = 0
                p[:] = 0
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            phat = dinv * p
            v = A @ phat
            matvecs += 1
            alpha = rho / np.vdot(rhat, v)
            s = r - alpha * v
            iters += 1
            if np.linalg.norm(s) / nf <= tol:
                x = x + alpha * phat
                hist.append(np.linalg.norm(s) / nf)
                done = True
                break
            shat = dinv * s
            t = A @ shat
            matvecs += 1
            tt = np.vdot(t, t)
            omega = np.vdot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha * phat + omega * shat
            r = s - omega * t
            rho_old = rho
            hist.append(np.linalg.norm(r) / nf)
            if hist[-1] <= tol:
                done = True
                break
        if not done:
            break
        # recursive residual says converged: the outer loop re-checks the true one
    rel = np.linalg.norm(f - A @ x) / nf
    return Result(x, 0 if rel <= tol else 1, iters, matvecs, rel, hist)


def bicgstab_l(A, f, l=4, tol=1e-8, max_matvec=20000, x0=None, precond="jacobi",
               on_cycle=None):
    """BiCGStab(l) of Sleijpen and Fokkema (ETNA 1, 1993), the paper's
    P-BiCGSTAB(8) family (Sec. 4, solver comparison table), on the
    right-Jacobi operator B = A D^-1.

    One cycle is l bi-conjugate gradient steps, each extending the chains
    u_0..u_{j+1} and r_0..r_{j+1} with u_{j+1} = B u_j and r_{j+1} = B r_j
    (2 products per step), followed by a minimal-residual step that picks
    gamma minimising ||r_0 - sum_{j>=1} gamma_j r_j|| (modified Gram-Schmidt
    on r_1..r_l, as in the original paper) and updates
        x += sum_j gamma_j r_{j-1},  r_0 -= sum_j gamma_j r_j,
        u_0 -= sum_j gamma_j u_j,    omega = gamma_l.
    Shadow residual r~ = r_0 of the (re)start.  On breakdown (rho or
    sigma zero) the method restarts from the true residual.  Convergence is
    tested on the recursive residual after each cycle and confirmed with the
    true residual.

    on_cycle(r_list, gamma): optional hook called before each minimal-residual
    update with the l+1 residual-chain vectors r_0..r_l (as formed by the
    bi-conjugate gradient part) and the chosen gamma[1..l]."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.size
    dinv = _dinv(A, precond)

    def B(z):
        return A @ (dinv * z)

    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    u_sol = x / dinv                      # iterate of B u = f
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return Result(np.zeros(n, dtype=np.complex128), 0, 0, 0, 0.0, [])
    matvecs, cycles, hist = 0, 0, []
    converged = False
    while not converged and matvecs < max_matvec:
        r = [f - B(u_sol)] + [None] * l
        matvecs += 1
        hist.append(np.linalg.norm(r[0]) / nf)
        if hist[-1] <= tol:
            converged = True
            break
        rt = r[0].copy()
        uu = [np.zeros(n, dtype=np.complex128)] + [None] * l
        rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
        breakdown = False
        while matvecs + 2 * l <= max_matvec:
            rho0 = -omega * rho0
            for j in range(l):
                rho1 = np.vdot(rt, r[j])
                if rho0 == 0 or rho1 == 0:
                    breakdown = True
                    break
                beta = alpha * rho1 / rho0
                rho0 = rho1
                for i in range(j + 1):
                    uu[i] = r[i] - beta * uu[i]
                uu[j + 1] = B(uu[j])
                sigma = np.vdot(rt, uu[j + 1])
                if sigma == 0:
                    breakdown = True
                    break
                alpha = rho0 / sigma
                for i in range(j + 1):
                    r[i] = r[i] - alpha * uu[i + 1]
                r[j + 1] = B(r[j])
                u_sol = u_sol + alpha * uu[0]
                matvecs += 2
            if breakdown:
                break
            # minimal-residual part: modified Gram-Schmidt on r_1..r_l
            q = [None] + [r[j].copy() for j in range(1, l + 1)]
            tau = np.zeros((l + 1, l + 1), dtype=np.complex128)
            sig = np.zeros(l + 1)
            gp = np.zeros(l + 1, dtype=np.complex128)
            for j in range(1, l + 1):
                for i in range(1, j):
                    tau[i, j] = np.vdot(q[i], q[j]) / sig[i]
                    q[j] = q[j] - tau[i, j] * q[i]
                sig[j] = np.vdot(q[j], q[j]).real
                if sig[j] == 0.0:
                    breakdown = True
                    break
                gp[j] = np.vdot(q[j], r[0]) / sig[j]
            if breakdown:
                break
            # back substitution: R gamma = gamma' with R unit upper triangular (tau)
            g = np.zeros(l + 1, dtype=np.complex128)
            for j in range(l, 0, -1):
                g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, l + 1))
            if on_cycle is not None:
                on_cycle([v.copy() for v in r], g[1:].copy())
            omega = g[l]
            u_sol = u_sol + sum(g[j] * r[j - 1] for j in range(1, l + 1))
            r0 = r[0] - sum(g[j] * r[j] for j in range(1, l + 1))
            uu[0] = uu[0] - sum(g[j] * uu[j] for j in range(1, l + 1))
            r[0] = r0
            cycles += 1
            hist.append(np.linalg.norm(r[0]) / nf)
            if hist[-1] <= tol:
                break
            if omega == 0:
                breakdown = True
                break
        if matvecs + 2 * l > max_matvec and not (hist and hist[-1] <= tol):
            break
        # recursive residual converged or breakdown: the loop restarts from the
        # true residual, which also confirms convergence
    x = dinv * u_sol
    rel = np.linalg.norm(f - A @ x) / nf
    return Result(x, 0 if rel <= tol else 1, cycles, matvecs, rel, hist)


def tfqmr(A, f, tol=1e-8, max_matvec=20000, x0=None, precond="jacobi", max_steps=None):
    """Transpose-free QMR of Freund (SIAM J. Sci. Comput. 14, 1993), the
    paper's P-tfQMR (Sec. 4, solver comparison table), on the right-Jacobi
    operator B = A D^-1 (iterate u of B u = f, x = D^-1 u).

    Half-steps m = 0, 1, 2, ...: on even m the CGS direction advances
    (alpha = rho / r*^H v, u_next = u - alpha v); on every m the quasi-residual
    w and the QMR direction d update and the smoothed iterate moves by
    eta d, with theta = ||w|| / tau, c = 1 / sqrt(1 + theta^2), tau = tau theta c,
    eta = c^2 alpha; on odd m the next CGS direction is built from
    rho = r*^H w, beta = rho / rho_old.  Shadow vector r* = r0.  The
    quasi-residual bound tau sqrt(m + 1) <= tol ||f|| stops the iteration,
    which is confirmed (or restarted) with the true residual; a zero
    r*^H v or rho restarts from the true residual as well.  max_steps caps
    the half-steps (for comparing iterates)."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.size
    dinv = _dinv(A, precond)

    def B(z):
        return A @ (dinv * z)

    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    u_sol = x / dinv
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return Result(np.zeros(n, dtype=np.complex128), 0, 0, 0, 0.0, [])
    matvecs, steps, hist = 0, 0, []
    converged = False
    while not converged and matvecs < max_matvec:
        r0 = f - B(u_sol)
        matvecs += 1
        hist.append(np.linalg.norm(r0) / nf)
        if hist[-1] <= tol:
            converged = True
            break
        rstar = r0.copy()
        w = r0.copy()
        u = r0.copy()
        v = B(u)
        matvecs += 1
        uhat = v.copy()                       # B u
        d = np.zeros(n, dtype=np.complex128)
        theta, eta = 0.0, 0.0 + 0.0j
        tau = np.linalg.norm(r0)
        rho = np.vdot(rstar, r0)
        alpha = 0.0 + 0.0j
        u_next = None
        m = 0
        restart = False
        while matvecs < max_matvec:
            if m % 2 == 0:
                sigma = np.vdot(rstar, v)
                if sigma == 0:
                    restart = True
                    break
                alpha = rho / sigma
                u_next = u - alpha * v
            w = w - alpha * uhat
            d = u + (theta ** 2 / alpha) * eta * d
            theta = np.linalg.norm(w) / tau
            c = 1.0 / np.sqrt(1.0 + theta ** 2)
            tau = tau * theta * c
            eta = c * c * alpha
            u_sol = u_sol + eta * d
            steps += 1
            if max_steps is not None and steps >= max_steps:
                break
            if tau * np.sqrt(m + 1) <= tol * nf:
                break                         # the outer loop checks the true residual
            if m % 2 == 1:
                rho_new = np.vdot(rstar, w)
                if rho == 0:
                    restart = True
                    break
                beta = rho_new / rho
                rho = rho_new
                u = w + beta * u
                v_part = beta * uhat + beta * beta * v
                uhat = B(u)
                matvecs += 1
                v = v_part + uhat
            else:
                u = u_next
                uhat = B(u)
                matvecs += 1
            m += 1
        if (not restart and matvecs >= max_matvec) or (max_steps is not None and steps >= max_steps):
            break
    x = dinv * u_sol
    rel = np.linalg.norm(f - A @ x) / nf
    return Result(x, 0 if rel <= tol else 1, steps, matvecs, rel, hist)
