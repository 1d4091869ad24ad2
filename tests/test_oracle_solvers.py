"""Pins of the oracle's solvers: dense brute force, exact special cases,
Krylov minimisation properties, symmetry/reciprocity and power balance."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import direct, fem, helmholtz as H, krylov

pytestmark = pytest.mark.cpu


def _system(elems, cfg=1, freq=137.0, eta=False):
    mesh = W.box_mesh(*elems)
    wl = W.workload(cfg, elems=elems)
    rng = np.random.default_rng(5)
    et = rng.uniform(0, 0.02, mesh["n_elems"]) if eta else None
    S = H.System(mesh, wl["beta"], et)
    k = W.wavenumber(freq)
    return mesh, S, S.operator(k), k, wl


@pytest.mark.parametrize("elems", [(1, 1, 1), (2, 2, 2), (4, 3, 2)])
def test_p6_brute_force_dense(elems):
    mesh, S, A, k, wl = _system(elems)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    x = np.linalg.solve(A.toarray(), f)
    for y in (direct.banded_solve(A, f), direct.banded_solve(A, f, mesh["xyz"]),
              direct.SparseLU(A).solve(f)):
        assert np.linalg.norm(y - x) <= 1e-12 * np.linalg.norm(x)
    kappa = np.linalg.cond(A.toarray())
    for res in (krylov.gmres(A, f, m=30, tol=1e-12), krylov.bicgstab(A, f, tol=1e-12)):
        assert res.status == 0 and res.relres <= 1e-12
        assert np.linalg.norm(res.x - x) <= 10 * kappa * 1e-12 * np.linalg.norm(x)


def test_p6_workload0_dense_and_krylov():
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0]))
    f = S.load(wl["g"])
    Ad = A.toarray()
    x = np.linalg.solve(Ad, f)
    xb = direct.banded_solve(A, f, wl["mesh"]["xyz"])
    assert np.linalg.norm(xb - x) <= 1e-12 * np.linalg.norm(x)
    kappa = np.linalg.cond(Ad)
    for res in (krylov.gmres(A, f, m=30, tol=1e-8), krylov.bicgstab(A, f, tol=1e-8)):
        assert res.status == 0 and res.relres <= 1e-8
        assert np.linalg.norm(res.x - x) <= kappa * 1e-8 * np.linalg.norm(x)
        assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)


def test_banded_lu_pivots():
    # a band matrix that needs row interchanges (zero leading diagonal entries)
    rng = np.random.default_rng(3)
    n, kl, ku = 40, 3, 2
    A = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for j in range(max(0, i - kl), min(n, i + ku + 1)):
            A[i, j] = rng.standard_normal() + 1j * rng.standard_normal()
    A[np.arange(n), np.arange(n)] = 0.0
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = direct.BandedLU(sp.csr_matrix(A)).solve(b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b) * np.linalg.cond(A)


def test_jacobi_on_diagonal_system_is_exact_in_one_step():
    # right-Jacobi makes A D^-1 = I for diagonal A: one Krylov step solves it
    rng = np.random.default_rng(2)
    d = rng.standard_normal(50) + 1j * rng.standard_normal(50) + 3.0
    A = sp.diags(d).tocsr()
    f = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    g = krylov.gmres(A, f, m=10, tol=1e-14)
    assert g.iters == 1 and np.allclose(g.x, f / d, rtol=1e-14)
    b = krylov.bicgstab(A, f, tol=1e-14)
    assert b.iters == 1 and np.allclose(b.x, f / d, rtol=1e-14)


def test_p7_power_balance():
    mesh, S, A, k, wl = _system((6, 4, 3), eta=True)
    f = S.load(wl["g"])
    p = direct.SparseLU(A).solve(f)
    lhs = np.imag(np.vdot(p, f))
    rhs = 0.0
    for w in range(6):
        rhs += k * wl["beta"][w].real * np.real(np.vdot(p, S.asm["B0"][w] @ p))
    Me = S.asm["Me"]
    pe = p[mesh["hex"]]
    rhs += k * k * np.sum(S.eta * np.real(np.einsum("ea,eab,eb->e", np.conj(pe), Me, pe)))
    assert lhs > 0 and rhs > 0
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_p8_complex_symmetry_and_reciprocity():
    mesh, S, A, k, wl = _system((5, 4, 3), eta=True)
    assert (A != A.T).nnz == 0
    lu = direct.SparseLU(A)
    i, j = 7, 83
    ei = np.zeros(S.n, complex); ei[i] = 1
    ej = np.zeros(S.n, complex); ej[j] = 1
    xi, xj = lu.solve(ei), lu.solve(ej)
    assert abs(xi[j] - xj[i]) <= 1e-12 * abs(xi[j])
    # adjoint solve A^H lam = s equals conj(A^-1 conj(s))
    rng = np.random.default_rng(4)
    s = rng.standard_normal(S.n) + 1j * rng.standard_normal(S.n)
    lam = np.linalg.solve(A.toarray().conj().T, s)
    assert np.allclose(lam, np.conj(lu.solve(np.conj(s))), rtol=1e-11, atol=1e-14 * abs(lam).max())


def test_p9_real_special_case():
    mesh = W.box_mesh(6, 4, 3)
    S = H.System(mesh, np.zeros(6, complex))
    A = S.operator(W.wavenumber(111.0))
    rng = np.random.default_rng(9)
    f = rng.standard_normal(S.n).astype(complex)
    for x in (direct.SparseLU(A).solve(f), krylov.gmres(A, f, m=20, tol=1e-10).x,
              krylov.bicgstab(A, f, tol=1e-10).x, direct.banded_solve(A, f)):
        assert np.abs(x.imag).max() <= 1e-15 * np.abs(x).max()


def test_p10_gmres_exactness_and_minimal_residual():
    mesh, S, A, k, wl = _system((2, 1, 1))
    n = S.n
    rng = np.random.default_rng(8)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = krylov.gmres(A, f, m=n, tol=1e-13)
    assert r.status == 0 and r.iters <= n
    # one cycle: each Givens residual estimate equals the least-squares minimum over K_j
    mesh, S, A, k, wl = _system((4, 3, 2))
    f = S.load(wl["g"]) + 0.1
    m = 8
    res = krylov.gmres(A, f, m=m, tol=1e-16, max_matvec=m + 1, record_cycles=True)
    est = np.array(res.cycles[0])
    dinv = 1.0 / A.diagonal()
    AD = A @ sp.diags(dinv)
    Kry = [f / np.linalg.norm(f)]
    for j in range(m):
        v = AD @ Kry[-1]
        Kry.append(v / np.linalg.norm(v))
    nf = np.linalg.norm(f)
    for j in range(1, m + 1):
        Q, _ = np.linalg.qr(np.stack(Kry[:j], axis=1))
        y, *_ = np.linalg.lstsq(AD @ Q, f, rcond=None)
        best = np.linalg.norm(f - AD @ (Q @ y)) / nf
        assert abs(est[j - 1] - best) <= 1e-10 * max(best, 1e-300) + 1e-14
    assert np.all(np.diff(est) <= 1e-15)


def test_bicgstab_restarts_from_true_residual_and_caps():
    mesh, S, A, k, wl = _system((4, 3, 2))
    f = S.load(wl["g"])
    r = krylov.bicgstab(A, f, tol=1e-8, max_matvec=5)
    assert r.status == 1 and r.matvecs <= 5
    r = krylov.gmres(A, f, m=5, tol=1e-8, max_matvec=3)
    assert r.status == 1 and r.matvecs <= 4


def test_bicgstab_l1_equals_scipy_bicgstab_iterates():
    """BiCGStab(1) is van der Vorst's BiCGStab: its iterate after k cycles is
    SciPy's right-preconditioned BiCGStab iterate after k iterations (same
    shadow residual r~ = r0 = f)."""
    import scipy.sparse.linalg as spla
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0])).tocsr()
    f = S.load(wl["g"])
    f = f / np.linalg.norm(f)
    dinv = 1.0 / A.diagonal()
    M = spla.LinearOperator(A.shape, matvec=lambda z: dinv * z, dtype=np.complex128)
    its = []
    spla.bicgstab(A, f, rtol=1e-300, atol=0.0, maxiter=8, M=M, callback=lambda xk: its.append(xk.copy()))
    assert len(its) == 8
    for k in (1, 2, 5, 8):
        res = krylov.bicgstab_l(A, f, l=1, tol=1e-300, max_matvec=1 + 2 * k)
        assert res.iters == k and res.matvecs == 1 + 2 * k
        assert np.linalg.norm(res.x - its[k - 1]) <= 1e-9 * np.linalg.norm(its[k - 1]), k


@pytest.mark.parametrize("n,l", [(8, 2), (8, 4), (7, 2), (9, 4), (8, 8)])
def test_bicgstab_l_finite_termination(n, l):
    """Without breakdown the bi-conjugate gradient part terminates after n
    steps, so ceil(n / l) cycles solve an n x n system to rounding level."""
    rng = np.random.default_rng(n * 10 + l)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = sp.csr_matrix(G + G.T + 4 * n * np.eye(n))
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    cyc = -(-n // l)
    res = krylov.bicgstab_l(A, f, l=l, tol=1e-300, max_matvec=1 + 2 * l * cyc)
    x = np.linalg.solve(A.toarray(), f)
    assert res.iters == cyc
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_bicgstab_l_chain_and_minimal_residual():
    """Each cycle's residual chain satisfies r_j = B r_{j-1} (B = A D^-1), and
    gamma minimises ||r_0 - sum_j gamma_j r_j|| (checked by least squares)."""
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0])).tocsr()
    f = S.load(wl["g"])
    dinv = 1.0 / A.diagonal()
    seen = []

    def hook(r, g):
        seen.append(1)
        for j in range(1, len(r)):
            Br = A @ (dinv * r[j - 1])
            assert np.linalg.norm(r[j] - Br) <= 1e-9 * np.linalg.norm(Br)
        R = np.stack(r[1:], axis=1)
        gl, *_ = np.linalg.lstsq(R, r[0], rcond=None)
        assert np.linalg.norm(g - gl) <= 1e-6 * np.linalg.norm(gl)
        assert (np.linalg.norm(r[0] - R @ g)
                <= (1 + 1e-10) * np.linalg.norm(r[0] - R @ gl) + 1e-300)

    for l in (2, 4):
        seen.clear()
        krylov.bicgstab_l(A, f, l=l, tol=1e-300, max_matvec=1 + 2 * l * 5, on_cycle=hook)
        assert len(seen) == 5


@pytest.mark.parametrize("l", [1, 2, 4, 8])
def test_bicgstab_l_converges_to_direct_solution(l):
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0]))
    f = S.load(wl["g"])
    x = direct.SparseLU(A).solve(f)
    res = krylov.bicgstab_l(A, f, l=l, tol=1e-8, max_matvec=20000)
    assert res.status == 0 and res.relres <= 1e-8
    assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_tfqmr_equals_scipy_tfqmr_iterates(precond):
    """The oracle's transpose-free QMR follows Freund's recurrences: its
    iterate after k half-steps is SciPy's unpreconditioned TFQMR iterate on
    the same operator (A, or the column-scaled A D^-1 with x = D^-1 y)."""
    import scipy.sparse.linalg as spla
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0])).tocsr()
    f = S.load(wl["g"])
    f = f / np.linalg.norm(f)
    dinv = 1.0 / A.diagonal() if precond == "jacobi" else np.ones(A.shape[0], dtype=complex)
    Bm = (A @ sp.diags(dinv)).tocsr()
    its = []
    spla.tfqmr(Bm, f, rtol=1e-300, atol=0.0, maxiter=9, callback=lambda xk: its.append(xk.copy()))
    assert len(its) == 9
    for k in (1, 2, 3, 6, 9):
        res = krylov.tfqmr(A, f, tol=1e-300, max_steps=k, precond=precond)
        assert res.iters == k
        ref = dinv * its[k - 1]
        assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref), k


@pytest.mark.parametrize("n", [5, 8])
def test_tfqmr_finite_termination(n):
    """After 2n half-steps the underlying CGS residual vanishes, and so does
    the quasi-residual: the iterate is the exact solution of an n x n system."""
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = sp.csr_matrix(G + G.T + 4 * n * np.eye(n))
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    res = krylov.tfqmr(A, f, tol=1e-300, max_steps=2 * n)
    x = np.linalg.solve(A.toarray(), f)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_tfqmr_converges_to_direct_solution():
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0]))
    f = S.load(wl["g"])
    x = direct.SparseLU(A).solve(f)
    res = krylov.tfqmr(A, f, tol=1e-8, max_matvec=20000)
    assert res.status == 0 and res.relres <= 1e-8
    assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)


def test_row_block_operator_is_bitwise_the_csr_product():
    """The threaded product used to time the oracle on all host cores gives
    the same bits as A @ x, so the timed solver takes the same iterates."""
    import workloads as W
    from oracle import helmholtz as H, krylov
    from oracle.parallel import RowBlockOperator
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(100.0)).tocsr()
    f = S.load(wl["g"])
    rng = np.random.default_rng(3)
    x = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    for t in (1, 3, 8):
        B = RowBlockOperator(A, t)
        assert np.array_equal(B @ x, A @ x)
        assert np.array_equal(B.diagonal(), A.diagonal())
        B.close()
    B = RowBlockOperator(A, 4)
    r1 = krylov.bicgstab(A, f, tol=1e-8)
    r2 = krylov.bicgstab(B, f, tol=1e-8)
    B.close()
    assert r1.iters == r2.iters and np.array_equal(r1.x, r2.x)
