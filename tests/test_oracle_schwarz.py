"""Pins of the oracle's Schwarz decomposition: the trivial partition is the
global solve, the exact interface fixed point reproduces the global solution
(by a dense solve of the interface system, independent of the iteration's
convergence), the transmission identity holds there, and the partition
covers every element and wall face once."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, helmholtz as H, schwarz

pytestmark = pytest.mark.cpu


def _global(elems, cfg=1, freq=130.0, eta=False):
    wl = W.workload(cfg, elems=elems)
    mesh = wl["mesh"]
    rng = np.random.default_rng(2)
    et = rng.uniform(0, 0.02, mesh["n_elems"]) if eta else None
    S = H.System(mesh, wl["beta"], et)
    k = W.wavenumber(freq)
    A = S.operator(k)
    g = wl["g"] if np.any(wl["g"]) else np.zeros(mesh["n_nodes"], complex)
    f = S.load(g) + 0.01 * (rng.standard_normal(mesh["n_nodes"]) + 1j * rng.standard_normal(mesh["n_nodes"]))
    return wl, mesh, et, k, A, f


def test_partition_covers_elements_and_faces_once():
    mesh = W.box_mesh(7, 5, 4)
    parts = (3, 2, 2)
    subs = schwarz.partition(mesh, parts)
    ne = 0
    nwall = 0
    for s in range(len(subs)):
        L = schwarz.local_mesh(mesh, parts, s)
        ne += L["n_elems"]
        nwall += int(np.sum(L["bface_tag"] < 6))
        # local node coordinates are the global ones
        assert np.allclose(L["xyz"], mesh["xyz"][L["l2g"]])
    assert ne == mesh["n_elems"]
    assert nwall == mesh["bface"].shape[0]


def test_trivial_partition_is_the_global_solve():
    wl, mesh, et, k, A, f = _global((6, 4, 3), eta=True)
    D = schwarz.Schwarz(mesh, (1, 1, 1), wl["beta"], et, k, f)
    assert len(D.pairs) == 0
    u = D.glue(D.local_solve([]))
    x = direct.SparseLU(A).solve(f)
    assert np.linalg.norm(u - x) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("parts,alpha", [((2, 1, 1), None), ((2, 2, 1), None), ((2, 2, 2), 0.7 + 2.0j),
                                         ((2, 2, 2), (0.7 + 2.0j, 3.1 + 0.4j)), ((3, 1, 2), (0.2 + 5.0j, 1.5 + 1.5j))])
def test_interface_fixed_point_is_the_global_solution(parts, alpha):
    wl, mesh, et, k, A, f = _global((6, 4, 4), eta=True)
    D = schwarz.Schwarz(mesh, parts, wl["beta"], et, k, f, alpha=alpha)
    IB, c, split = D.interface_matrix()
    lam = split(np.linalg.solve(IB, c))
    us = D.local_solve(lam)
    u = D.glue(us)
    x = direct.SparseLU(A).solve(f)
    assert np.linalg.norm(u - x) <= 1e-10 * np.linalg.norm(x)
    # duplicated interface values agree, and lam_st + lam_ts = (a_lo + a_hi) M_G u_G
    for i, p in enumerate(D.pairs):
        assert np.allclose(us[p["s"]][p["ins"]], us[p["t"]][p["int"]], rtol=1e-10, atol=1e-12 * abs(x).max())
        j = D.index[(p["t"], p["s"])]
        lhs = lam[i] + lam[j]
        rhs = (D.a_lo + D.a_hi) * (p["MG"] @ us[p["s"]][p["ins"]])
        assert np.linalg.norm(lhs - rhs) <= 1e-9 * np.linalg.norm(rhs)


def test_imaginary_alpha_iteration_is_nonexpansive():
    # With T = alpha M_G and alpha purely imaginary the Robin-to-Robin map is
    # non-expansive (the local Dirichlet-to-Neumann maps of the damped cavity
    # have a non-negative imaginary part), so every eigenvalue of the
    # iteration operator B lies in the closed unit disc.
    wl, mesh, et, k, A, f = _global((6, 4, 4), freq=90.0)
    for parts in ((2, 1, 1), (2, 2, 1)):
        D = schwarz.Schwarz(mesh, parts, wl["beta"], et, k, f)
        IB, c, split = D.interface_matrix()
        ev = np.linalg.eigvals(np.eye(IB.shape[0]) - IB)
        assert np.abs(ev).max() <= 1 + 1e-10


def test_richardson_history_and_interface_gmres():
    from oracle import krylov
    wl, mesh, et, k, A, f = _global((8, 6, 4), freq=60.0)
    D = schwarz.Schwarz(mesh, (2, 2, 1), wl["beta"], et, k, f)
    u, lams, hist = D.richardson(20, A, f)
    assert np.all(np.isfinite(hist)) and hist[-1, 1] < hist[0, 1]
    op, c, split = D.interface_operator()
    r = krylov.gmres(op, c, m=40, tol=1e-11, max_matvec=2000, precond="none")
    assert r.status == 0
    u = D.glue(D.local_solve(split(r.x)))
    x = direct.SparseLU(A).solve(f)
    assert np.linalg.norm(u - x) <= 1e-8 * np.linalg.norm(x)
