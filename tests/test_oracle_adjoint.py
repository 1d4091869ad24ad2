"""Pin of the oracle's adjoint gradient against central finite differences."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint

pytestmark = pytest.mark.cpu

H_FD = 1e-6


def _fd(fun, x0, i, h=H_FD):
    xp = x0.copy(); xp[i] += h
    xm = x0.copy(); xm[i] -= h
    return (fun(xp) - fun(xm)) / (2 * h)


def _case(elems, nfreq, nrec, seed=1):
    mesh = W.box_mesh(*elems)
    wl = W.workload(4, elems=elems)
    rng = np.random.default_rng(seed)
    eta = rng.uniform(0, 0.02, mesh["n_elems"])
    nx, ny, nz = elems
    interior = [W.node_id(i, j, k, nx, ny) for k in range(1, nz) for j in range(1, ny) for i in range(1, nx)]
    rec = rng.choice(interior, size=min(nrec, len(interior)), replace=False)
    freqs = np.linspace(50, 200, nfreq)
    return mesh, wl["beta"], eta, freqs, wl["g"], rec


def test_p12_gradient_vs_central_fd_all_parameters_small_mesh():
    mesh, beta, eta, freqs, g, rec = _case((4, 3, 2), nfreq=2, nrec=4)
    J, db, de, _, _ = adjoint.gradient(mesh, beta, eta, freqs, g, rec)
    J0, _ = adjoint.energy(mesh, beta, eta, freqs, g, rec)
    assert abs(J - J0) <= 1e-13 * J

    def J_beta(v):
        b = v[0::2] + 1j * v[1::2]
        return adjoint.energy(mesh, b, eta, freqs, g, rec)[0]

    bv = np.stack([beta.real, beta.imag], axis=1).ravel()
    fd_b = np.array([_fd(J_beta, bv, i) for i in range(12)])
    assert np.linalg.norm(fd_b - db.ravel()) <= 1e-6 * np.linalg.norm(db)

    def J_eta(v):
        return adjoint.energy(mesh, beta, v, freqs, g, rec)[0]

    fd_e = np.array([_fd(J_eta, eta, i) for i in range(eta.size)])
    assert np.linalg.norm(fd_e - de) <= 1e-6 * np.linalg.norm(de)


@pytest.mark.slow
def test_p12_gradient_directional_workload0_size():
    mesh, beta, eta, freqs, g, rec = _case((20, 12, 10), nfreq=2, nrec=16, seed=3)
    J, db, de, _, _ = adjoint.gradient(mesh, beta, eta, freqs, g, rec)

    def J_eta(v):
        return adjoint.energy(mesh, beta, v, freqs, g, rec)[0]

    rng = np.random.default_rng(12)
    v = rng.standard_normal(eta.size)
    dd = (J_eta(eta + H_FD * v) - J_eta(eta - H_FD * v)) / (2 * H_FD)
    assert abs(dd - de @ v) <= 1e-6 * abs(de @ v)
    for i in rng.choice(eta.size, 4, replace=False):
        fd = _fd(J_eta, eta, i)
        assert abs(fd - de[i]) <= 1e-5 * np.abs(de).max()


def test_p12_gradient_vs_central_fd_tetrahedra():
    """The same pin on an unstructured tetrahedral (P1) mesh."""
    mesh = W.kuhn_tet_mesh(3, 2, 2)
    wl = W.workload(4, elems=(4, 3, 2))
    beta = wl["beta"]
    rng = np.random.default_rng(9)
    eta = rng.uniform(0, 0.02, mesh["n_elems"])
    rec = rng.choice(mesh["n_nodes"], size=5, replace=False)
    g = np.zeros(mesh["n_nodes"], dtype=complex)
    pn = W.patch_nodes(mesh)
    g[pn] = rng.standard_normal(pn.size) + 1j * rng.standard_normal(pn.size)
    freqs = np.array([80.0, 170.0])
    J, db, de, _, _ = adjoint.gradient(mesh, beta, eta, freqs, g, rec)

    def J_beta(v):
        return adjoint.energy(mesh, v[0::2] + 1j * v[1::2], eta, freqs, g, rec)[0]

    bv = np.stack([beta.real, beta.imag], axis=1).ravel()
    fd_b = np.array([_fd(J_beta, bv, i) for i in range(12)])
    assert np.linalg.norm(fd_b - db.ravel()) <= 1e-6 * np.linalg.norm(db)

    def J_eta(v):
        return adjoint.energy(mesh, beta, v, freqs, g, rec)[0]

    fd_e = np.array([_fd(J_eta, eta, i) for i in range(eta.size)])
    assert np.linalg.norm(fd_e - de) <= 1e-6 * np.linalg.norm(de)
