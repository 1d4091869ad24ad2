"""Full-size checks at the benchmark's workload (160x96x80 box, 250 Hz,
1,264,977 unknowns) in the configuration bench.py times: sampled rows of
the sparse product against the oracle's rows, and the BiCGStab solve's
residual recomputed by the oracle's element-by-element operator."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import helmholtz as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c1():
    import paper_2112_00087_amd as P
    assert torch.cuda.is_available()
    wl = W.workload(1)
    model = P.Helmholtz(wl["mesh"], wl["beta"])
    model.set_frequency(wl["freqs"][0])
    yield wl, model
    model.close()


def test_spmv_sampled_rows_full_size(c1):
    wl, model = c1
    mesh = wl["mesh"]
    n = mesh["n_nodes"]
    nx, ny, nz = mesh["elems"]
    rng = np.random.default_rng(21)
    corners = [W.node_id(i, j, k, nx, ny) for i in (0, nx) for j in (0, ny) for k in (0, nz)]
    edges = [W.node_id(i, 0, 0, nx, ny) for i in (1, nx // 2, nx - 1)]
    rows = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), corners, edges,
                                     np.arange(n - 70, n), np.arange(0, 70)]))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = model.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    R = H.rows_of_operator(mesh, W.wavenumber(wl["freqs"][0]), wl["beta"], None, rows)
    yref = R @ x
    # Off-diagonal Q1 entries of these thin elements are small differences of
    # Gauss-point terms of the size of the diagonal, so assembly rounding scales
    # with the row's magnitude: bound by 1e-14 ||A_i||_1 max|x|.
    bound = 1e-14 * (abs(R) @ np.ones(n)) * np.abs(x).max()
    assert np.all(np.abs(y[rows] - yref) <= bound)


@pytest.mark.parametrize("method,l", [("bicgstab", 0), ("bicgstabl", 4), ("tfqmr", 0), ("gmres", 50)])
def test_bicgstab_full_size_residual_by_oracle(c1, method, l):
    wl, model = c1
    f = model.load(torch.as_tensor(wl["g"], device="cuda"))
    model.set_frequency(wl["freqs"][0])
    p, info = model.solve(f, method=method, restart=l or 30, tol=1e-8, max_matvec=100000)
    say(f"full-size {method}", info)
    assert info["status"] == 0
    p = p.cpu().numpy()
    fo = H.load_elementwise(wl["mesh"], wl["g"])
    Ap = H.apply_elementwise(wl["mesh"], W.wavenumber(wl["freqs"][0]), wl["beta"], None, p)
    rel = np.linalg.norm(fo - Ap) / np.linalg.norm(fo)
    say(f"  oracle relres {rel:.3e}")
    assert rel <= 1e-8
    assert abs(rel - info["relres_true"]) <= 1e-3 * rel


@pytest.fixture(scope="module", params=[5, 6])
def c5(request):
    """Unstructured workloads (48x32x32 Kuhn cells split into 1,179,648
    hexahedra, 1,302,753 nodes; 144x96x96 cells of 7,962,624 P1 tetrahedra,
    1,364,305 nodes; random node numbering) in the row numbering the
    unstructured bench leg times."""
    import paper_2112_00087_amd as P
    assert torch.cuda.is_available()
    wl = W.workload(request.param)
    model = P.Helmholtz(wl["mesh"], wl["beta"], order="rcm", sigma=256)
    model.set_frequency(wl["freqs"][0])
    yield wl, model
    model.close()


def test_unstructured_spmv_sampled_rows_full_size(c5):
    wl, model = c5
    mesh = wl["mesh"]
    n = mesh["n_nodes"]
    rng = np.random.default_rng(23)
    perm = model.layout()["perm"]
    # random rows, the first and last internal rows, and the longest rows
    rl = np.bincount((mesh["tet"] if "tet" in mesh else mesh["hex"]).ravel(), minlength=n)
    rows = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), perm[:70], perm[-70:],
                                     np.argsort(rl)[-50:]]))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = model.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    R = H.rows_of_operator(mesh, W.wavenumber(wl["freqs"][0]), wl["beta"], None, rows)
    yref = R @ x
    bound = 1e-14 * (abs(R) @ np.ones(n)) * np.abs(x).max()
    assert np.all(np.abs(y[rows] - yref) <= bound)


def test_unstructured_full_size_residual_by_oracle(c5):
    wl, model = c5
    f = model.load(torch.as_tensor(wl["g"], device="cuda"))
    p, info = model.solve(f, method="bicgstabl", restart=4, tol=1e-8, max_matvec=100000)
    say("full-size unstructured bicgstab(4)", wl["name"], info)
    assert info["status"] == 0
    p = p.cpu().numpy()
    fo = H.load_elementwise(wl["mesh"], wl["g"])
    Ap = H.apply_elementwise(wl["mesh"], W.wavenumber(wl["freqs"][0]), wl["beta"], None, p)
    rel = np.linalg.norm(fo - Ap) / np.linalg.norm(fo)
    say(f"  oracle relres {rel:.3e}")
    assert rel <= 1e-8
    assert abs(rel - info["relres_true"]) <= 1e-3 * rel


def test_schwarz_full_size_residual_by_oracle():
    """Workload 3 as configured: 200x120x100 box (2,456,421 unknowns) split
    4 x 3 x 2 = 24 subdomains of 50x40x50 elements, 150 Hz, interface GMRES
    in complex128 with the optimised two-sided coefficients, batched
    BiCGStab(4) local solves in complex64 with FP64 refinement (the bench's
    setting); the glued solution's residual recomputed by the oracle's
    element-by-element operator."""
    import paper_2112_00087_amd as P
    assert torch.cuda.is_available()
    wl = W.workload(3)
    model = P.Helmholtz(wl["mesh"], wl["beta"], parts=wl["parts"])
    model.set_frequency(wl["freqs"][0])
    f = model.load(torch.as_tensor(wl["g"], device="cuda"))
    p, info = model.solve(f, method="schwarz", tol=1e-8, restart=300, max_matvec=300, precision="mixed",
                          inner_tol=1e-10, dd_inner="bicgstabl", inner_restart=4)
    say("full-size schwarz", info)
    assert info["status"] == 0
    p = p.cpu().numpy()
    model.close()
    fo = H.load_elementwise(wl["mesh"], wl["g"])
    Ap = H.apply_elementwise(wl["mesh"], W.wavenumber(wl["freqs"][0]), wl["beta"], None, p)
    rel = np.linalg.norm(fo - Ap) / np.linalg.norm(fo)
    say(f"  oracle relres {rel:.3e}")
    assert rel <= 1e-8
    assert abs(rel - info["relres_true"]) <= 1e-3 * rel
