"""Pins of the oracle's matrix-free checkers against its assembled operator.

The full-size GPU tests judge residuals and sampled rows with three
matrix-free oracle functions (element-by-element product, face-by-face
load, and selected rows built only from the touching elements).  The
assembled ``System.operator`` / ``System.load`` they are compared with here
are themselves pinned by closed forms, the exact rigid-box modes, the 1-D
reduction and the plane-wave convergence (paper Sec. 3.2: the discrete
operator ``K - k^2 M + i k^2 M_eta + i k B_beta`` and the patch load).

Every wall carries a distinct complex admittance and the absorption field
is random, so a wrong face selection, a wrong sign or scale of the wall or
absorption term, a dropped term or a transposed element block changes the
result far beyond the 1e-14 bounds used here.
"""
import numpy as np
import pytest

import workloads as W
from oracle import helmholtz as H

pytestmark = pytest.mark.cpu

BETA = np.array([0.03 + 0.004j, 0.011 - 0.007j, 0.045 + 0.0j, 0.002 + 0.009j, 0.02 - 0.001j,
                 0.037 + 0.006j])


def _mesh(kind):
    if kind == "box":
        return W.box_mesh(9, 7, 5)
    if kind == "kuhn-hex":
        return W.kuhn_hex_mesh(3, 2, 2, seed=W.SEED + 17)
    return W.kuhn_tet_mesh(4, 3, 3, seed=W.SEED + 19)


def _cases():
    for kind in ("box", "kuhn-hex", "kuhn-tet"):
        for with_eta in (False, True):
            for k in (0.0, 3.7):
                yield kind, with_eta, k


def _inputs(mesh, with_eta, seed):
    rng = np.random.default_rng(seed)
    n = mesh["n_nodes"]
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    eta = rng.uniform(0.0, 0.05, mesh["n_elems"]) if with_eta else None
    return x, eta


@pytest.mark.parametrize("kind,with_eta,k", list(_cases()))
def test_apply_elementwise_equals_assembled_operator(kind, with_eta, k):
    mesh = _mesh(kind)
    x, eta = _inputs(mesh, with_eta, 5)
    A = H.System(mesh, BETA, eta).operator(k)
    y_ref = A @ x
    y = H.apply_elementwise(mesh, k, BETA, eta, x, chunk=37)   # several chunks, ragged last one
    scale = abs(A) @ abs(x)
    assert np.all(np.abs(y - y_ref) <= 1e-14 * scale)
    # the wall and absorption terms are really present at k > 0: dropping
    # either one moves the product far outside the bound
    if k > 0:
        y_nowall = H.apply_elementwise(mesh, k, np.zeros(6), eta, x)
        assert np.max(np.abs(y_nowall - y_ref) / scale) > 1e-6
        if with_eta:
            y_noeta = H.apply_elementwise(mesh, k, BETA, None, x)
            assert np.max(np.abs(y_noeta - y_ref) / scale) > 1e-6


@pytest.mark.parametrize("kind", ["box", "kuhn-hex", "kuhn-tet"])
def test_load_elementwise_equals_assembled_load(kind):
    mesh = _mesh(kind)
    rng = np.random.default_rng(7)
    n = mesh["n_nodes"]
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)     # nonzero everywhere: off-patch nodes must not load
    S = H.System(mesh, BETA)
    f_ref = S.load(g)
    f = H.load_elementwise(mesh, g)
    scale = abs(S.asm["Mpatch"]) @ abs(g)
    assert np.all(np.abs(f - f_ref) <= 1e-14 * scale)
    # only patch nodes carry load
    off = np.setdiff1d(np.arange(n), W.patch_nodes(mesh))
    assert np.all(f[off] == 0)
    assert np.count_nonzero(f) == W.patch_nodes(mesh).size


@pytest.mark.parametrize("kind,with_eta,k", list(_cases()))
def test_rows_of_operator_equal_assembled_rows(kind, with_eta, k):
    mesh = _mesh(kind)
    _, eta = _inputs(mesh, with_eta, 11)
    A = H.System(mesh, BETA, eta).operator(k)
    n = mesh["n_nodes"]
    rng = np.random.default_rng(13)
    # a random sample plus the extreme ids (corner / wall rows on the box)
    rows = np.unique(np.concatenate([rng.choice(n, size=min(n, 40), replace=False), [0, n - 1]]))
    R = H.rows_of_operator(mesh, k, BETA, eta, rows).toarray()
    Aref = A[rows].toarray()
    scale = np.abs(Aref).sum(1, keepdims=True)
    assert np.all(np.abs(R - Aref) <= 1e-14 * scale)
    # same sparsity: no entry outside the assembled pattern
    assert np.all((np.abs(R) > 0) <= (np.abs(Aref) > 0) | (np.abs(R) <= 1e-14 * scale))
