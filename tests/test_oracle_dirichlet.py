"""Pins of the oracle's Dirichlet source condition (paper Sec. 3.2: the
spectrum on the sun-roof opening is imposed as a Dirichlet condition) and of
its Galerkin least-squares stabilisation (the paper uses stabilised finite
elements without naming the scheme; GLS of Harari and Hughes, 1992, is the
reading), against what the mathematics fixes:

* the exact 1-D reduction with a Dirichlet end: a rigid box driven by a
  uniform prescribed pressure on its x- wall has p depending on x only, and
  the discrete solution is a * cos(theta (N - j)) with theta from the
  Galerkin dispersion relation; with GLS theta equals k h, so the nodes carry
  the continuum solution cos(k (L - x)) / cos(k L) exactly;
* the definition of the elimination on a general mesh: p = g on D, and the
  unmodified operator's free rows of A p vanish;
* the adjoint gradient through the eliminated system against central
  differences."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, direct, helmholtz as H


def _xminus_source(nx, ny, nz):
    mesh = W.box_mesh(nx, ny, nz)
    mesh["bface_src"] = (mesh["bface_tag"] == 0).astype(np.uint8)
    return mesh


@pytest.mark.parametrize("freq", [90.0, 130.0, 210.0])
@pytest.mark.parametrize("gls", [False, True])
def test_dirichlet_1d_reduction_exact(freq, gls):
    nx, ny, nz = 18, 12, 10               # cubes of edge 0.1 m
    mesh = _xminus_source(nx, ny, nz)
    h, L = 0.1, 1.8
    k = W.wavenumber(freq)
    S = H.System(mesh, np.zeros(6), dirichlet=True, gls=gls)
    assert abs(S.gls_h - (h if gls else 0.0)) <= 1e-15
    g0 = 0.7 - 0.4j
    g = np.zeros(S.n, dtype=np.complex128)
    g[S.D] = g0
    A = S.operator(k)
    p = direct.SparseLU(A).solve(S.load(g, k))
    x = mesh["xyz"][:, 0]
    j = np.rint(x / h)
    if gls:
        # nodally exact: the continuum solution with p(0) = g0, p'(L) = 0
        expect = g0 * np.cos(k * (L - x)) / np.cos(k * L)
    else:
        c = (1 - (k * h) ** 2 / 3) / (1 + (k * h) ** 2 / 6)
        th = np.arccos(c)
        expect = g0 * np.cos(th * (nx - j)) / np.cos(th * nx)
    assert np.max(np.abs(p - expect)) <= 1e-10 * np.max(np.abs(expect))
    # GLS moves the nodes onto the continuum solution, Galerkin does not
    cont = g0 * np.cos(k * (L - x)) / np.cos(k * L)
    if not gls:
        assert np.max(np.abs(p - cont)) > 1e-4 * np.max(np.abs(cont))


def test_gls_tau_limits():
    """tau k^2 -> -(kh)^2/12 for small kh and 0 at kh = 0 (the GLS correction
    vanishes as the mesh is refined)."""
    assert H.gls_tau_k2(0.0) == 0.0
    for t in (1e-2, 3e-2):
        assert abs(H.gls_tau_k2(t) + t * t / 12) <= 1e-3 * t * t / 12


@pytest.mark.parametrize("gls", [False, True])
def test_dirichlet_elimination_definition(gls):
    wl = W.workload(1, elems=(12, 8, 6))
    mesh = wl["mesh"]
    rng = np.random.default_rng(5)
    eta = rng.uniform(0, 0.02, mesh["n_elems"])
    S = H.System(mesh, wl["beta"], eta, dirichlet=True, gls=gls)
    assert S.D.size > 0
    k = W.wavenumber(170.0)
    A = S.operator(k)
    assert abs(A - A.T).max() == 0.0                  # still complex symmetric
    f = S.load(wl["g"], k)
    p = direct.SparseLU(A).solve(f)
    assert np.allclose(p[S.D], wl["g"][S.D], rtol=0, atol=1e-13 * np.abs(wl["g"]).max())
    Af = S.operator(k, eliminate=False)
    r = Af @ p
    free = np.ones(S.n, bool)
    free[S.D] = False
    scale = np.linalg.norm(Af[:, S.D] @ wl["g"][S.D])
    assert np.linalg.norm(r[free]) <= 1e-11 * scale
    # the Neumann reading of the same data is a different problem
    SN = H.System(mesh, wl["beta"], eta, gls=gls)
    pN = direct.SparseLU(SN.operator(k)).solve(SN.load(wl["g"]))
    assert np.linalg.norm(pN - p) > 1e-3 * np.linalg.norm(p)


@pytest.mark.parametrize("gls", [False, True])
def test_dirichlet_adjoint_gradient_vs_central_differences(gls):
    wl = W.workload(4, elems=(6, 4, 4))
    mesh = wl["mesh"]
    rng = np.random.default_rng(9)
    eta = rng.uniform(0, 0.02, mesh["n_elems"])
    freqs = [60.0, 140.0]
    rec = wl["receivers"][:4]
    J, db, de, _, _ = adjoint.gradient(mesh, wl["beta"], eta, freqs, wl["g"], rec, dirichlet=True, gls=gls)
    hstep = 1e-6

    def Jof(beta, et):
        return adjoint.energy(mesh, beta, et, freqs, wl["g"], rec, dirichlet=True, gls=gls)[0]

    for w in range(6):
        for part, d in ((0, 1.0), (1, 1j)):
            bp = wl["beta"].copy()
            bm = wl["beta"].copy()
            bp[w] += hstep * d
            bm[w] -= hstep * d
            fd = (Jof(bp, eta) - Jof(bm, eta)) / (2 * hstep)
            assert abs(fd - db[w, part]) <= 1e-6 * np.abs(db).max() + 1e-9 * abs(J), (w, part, fd, db[w, part])
    for e in rng.choice(mesh["n_elems"], 6, replace=False):
        ep = eta.copy()
        em = eta.copy()
        ep[e] += hstep
        em[e] -= hstep
        fd = (Jof(wl["beta"], ep) - Jof(wl["beta"], em)) / (2 * hstep)
        assert abs(fd - de[e]) <= 1e-6 * np.abs(de).max() + 1e-9 * abs(J), (e, fd, de[e])
