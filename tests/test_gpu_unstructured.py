"""GPU path on unstructured meshes (randomly numbered hexahedra from split
Kuhn tetrahedra, and the Kuhn tetrahedra themselves as P1 elements) under
each internal row numbering: the caller's, reverse Cuthill-McKee, and either
with the length sort of the sliced-ELL rows.
Vectors cross the C ABI in the mesh's numbering, so every result is compared
with the oracle element by element in that numbering."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, direct, helmholtz as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ORDERS = [("given", 0), ("rcm", 0), ("rcm", 256), ("given", 1024)]
WL = {"hex": 5, "tet": 6}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2112_00087_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return pkg


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.complex128), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


# (16, 12, 10) hexahedral and (40, 30, 30) tetrahedral cells: 50k and 39k
# nodes, so the caller's random numbering has column offsets beyond int16 and
# the split form falls back to int32 columns
@pytest.mark.parametrize("order,sigma", ORDERS)
@pytest.mark.parametrize("kind,cells,with_eta", [("hex", (2, 2, 1), False), ("hex", (5, 4, 3), True),
                                                 ("hex", (10, 8, 6), False), ("hex", (16, 12, 10), False),
                                                 ("tet", (4, 3, 3), False), ("tet", (12, 8, 8), True),
                                                 ("tet", (40, 30, 30), False)])
def test_unstructured_spmv_diag_load_parity(P, kind, cells, with_eta, order, sigma):
    say("unstructured spmv parity", kind, cells, with_eta, order, sigma)
    wl = W.workload(WL[kind], elems=cells)
    mesh = wl["mesh"]
    rng = np.random.default_rng(11)
    eta = rng.uniform(0, 0.02, mesh["n_elems"]) if with_eta else None
    S = H.System(mesh, wl["beta"], eta)
    model = P.Helmholtz(mesh, wl["beta"], eta, order=order, sigma=sigma)
    n = mesh["n_nodes"]
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for f in (0.0, 250.0):
        k = W.wavenumber(f)
        A = S.operator(k)
        model.set_frequency(f)
        y = _np(model.apply(_t(x)))
        yref = A @ x
        bound = 1e-14 * (abs(A) @ np.abs(x)) + 1e-300
        assert np.all(np.abs(y - yref) <= bound), (f, np.max(np.abs(y - yref) / bound))
        d = _np(model.diag())
        mag = (np.abs(S.asm["K"].diagonal()) + k * k * np.abs(S.asm["M"].diagonal())
               + (k * k * np.abs(S.Meta.diagonal()) if S.Meta is not None else 0.0)
               + k * np.abs(S.Bbeta.diagonal()))
        assert np.all(np.abs(d - A.diagonal()) <= 1e-14 * mag)
    f = _np(model.load(_t(wl["g"])))
    fref = S.load(wl["g"])
    # the load is a sparse product with the patch mass (entries summed from
    # face terms in another order): the product's rounding bound, as above
    bound = 1e-14 * (abs(S.asm["Mpatch"]) @ np.abs(wl["g"])) + 1e-300
    assert np.all(np.abs(f - fref) <= bound), np.max(np.abs(f - fref) / bound)
    model.close()


def test_unstructured_layout(P):
    """The internal numbering is a permutation; reverse Cuthill-McKee narrows
    the band of the randomly numbered mesh, and the length sort cuts the
    sliced-ELL padding (each 64-row slice is as wide as its longest row)."""
    wl = W.workload(5, elems=(10, 8, 6))
    mesh = wl["mesh"]
    n = mesh["n_nodes"]
    out = {}
    for order, sigma in ORDERS:
        m = P.Helmholtz(mesh, wl["beta"], order=order, sigma=sigma)
        lay = m.layout()
        nnz = m.sizes()["nnz"]
        assert np.array_equal(np.sort(lay["perm"]), np.arange(n))
        assert np.array_equal(lay["perm"], P.node_order(mesh, order, sigma))
        assert lay["slots"] >= nnz
        out[(order, sigma)] = (lay["slots"] / nnz, lay["bandwidth"])
        m.close()
    say("  padding, bandwidth:", out)
    assert out[("rcm", 0)][1] < out[("given", 0)][1] / 10
    # rows of 12 to 75 entries: unsorted slices are padded to near the
    # maximum, sorted ones to near their own length
    assert out[("given", 0)][0] > 2.0
    assert out[("rcm", 256)][0] < 0.5 * out[("given", 0)][0]
    assert out[("given", 1024)][0] < 0.5 * out[("given", 0)][0]


@pytest.fixture(scope="module", params=["hex", "tet"])
def u1(P, request):
    cells = (10, 8, 6) if request.param == "hex" else (30, 20, 20)
    wl = W.workload(WL[request.param], elems=cells)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0]))
    f = S.load(wl["g"])
    x = direct.SparseLU(A).solve(f)
    return dict(wl=wl, A=A, f=f, x=x, kind=request.param)


@pytest.mark.parametrize("order,sigma", [("given", 0), ("rcm", 256)])
@pytest.mark.parametrize("method,precision,restart", [("bicgstab", "fp64", 0), ("tfqmr", "fp64", 0),
                                                      ("gmres", "fp64", 50), ("bicgstabl", "fp64", 4),
                                                      ("tfqmr", "mixed", 0)])
def test_unstructured_solve_matches_oracle(P, u1, order, sigma, method, precision, restart):
    say("unstructured solve", u1["kind"], order, sigma, method, precision)
    wl = u1["wl"]
    m = P.Helmholtz(wl["mesh"], wl["beta"], order=order, sigma=sigma)
    m.set_frequency(wl["freqs"][0])
    kw = dict(restart=restart) if restart else {}
    if precision == "mixed":
        kw["inner_tol"] = 1e-2      # complex64 inner solves stall near 1e-3 on this indefinite system
    p, info = m.solve(_t(u1["f"]), method=method, precision=precision, tol=1e-8, max_matvec=50000, **kw)
    p = _np(p)
    rel = H.relres(u1["A"], p, u1["f"])
    err = np.linalg.norm(p - u1["x"]) / np.linalg.norm(u1["x"])
    say(f"  info={info} oracle relres={rel:.3e} relerr={err:.3e}")
    assert info["status"] == 0 and rel <= 1e-8 and err <= 1e-6
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel + 1e-15
    m.close()


@pytest.mark.parametrize("kind", ["hex", "tet"])
@pytest.mark.parametrize("method,precision", [("tfqmr", "fp64"), ("bicgstabl", "fp64"), ("gmres", "mixed")])
def test_unstructured_sweep_matches_oracle(P, kind, method, precision):
    say("unstructured sweep", kind, method, precision)
    wl = W.workload(WL[kind], elems=(6, 4, 4) if kind == "hex" else (12, 8, 8))
    mesh = wl["mesh"]
    freqs = np.array([40.0, 120.0, 200.0, 260.0, 300.0])
    S = H.System(mesh, wl["beta"])
    f = S.load(wl["g"])
    F = np.stack([f * (1.0 + 0.1 * j) for j in range(freqs.size)], axis=1)
    model = P.Helmholtz(mesh, wl["beta"], order="rcm", sigma=256)
    Pg, infos = model.solve_sweep(freqs, _t(F), method=method, restart=4 if method == "bicgstabl" else 60,
                                  tol=1e-10, precision=precision, max_matvec=50000)
    Pg = Pg.cpu().numpy()
    for j, fr in enumerate(freqs):
        A = S.operator(W.wavenumber(fr))
        x = direct.SparseLU(A).solve(F[:, j])
        rel = H.relres(A, Pg[:, j], F[:, j])
        err = np.linalg.norm(Pg[:, j] - x) / np.linalg.norm(x)
        assert infos[j]["status"] == 0, (j, infos[j])
        assert rel <= 1e-10 * 1.01, (j, rel)
        assert err <= 1e-6, (j, fr, err)
    model.close()


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_unstructured_adjoint_gradient_matches_oracle(P, kind):
    """Adjoint gradient with an absorption field under the reordered
    numbering: element- and wall-indexed results stay in the mesh's order."""
    say("unstructured adjoint", kind)
    wl = W.workload(WL[kind], elems=(4, 3, 3) if kind == "hex" else (8, 6, 6))
    mesh = wl["mesh"]
    rng = np.random.default_rng(5)
    eta = rng.uniform(0.0, 0.02, mesh["n_elems"])
    rec = np.sort(rng.choice(mesh["n_nodes"], size=12, replace=False)).astype(np.int64)
    freqs = np.array([90.0, 170.0])
    model = P.Helmholtz(mesh, wl["beta"], eta, order="rcm", sigma=256)
    f = model.load(_t(wl["g"]))
    rt = torch.as_tensor(rec, device="cuda")
    deta = torch.zeros(model.ne, dtype=torch.float64, device="cuda")
    db = np.zeros((6, 2))
    J = 0.0
    for fr in freqs:
        model.set_frequency(fr)
        p, info = model.solve(f, method="gmres", tol=1e-12, restart=60, max_matvec=200000)
        assert info["status"] == 0, info
        J += float((p[rt].abs() ** 2).sum())
        g = torch.zeros_like(p)
        g[rt] = p[rt]
        _, dbf, info = model.solve_adjoint(p, g, dJ_deta=deta, method="gmres", tol=1e-12, restart=60,
                                           max_matvec=200000)
        assert info["status"] == 0, info
        db += dbf
    Jo, dbo, deo, _, _ = adjoint.gradient(mesh, wl["beta"], eta, freqs, wl["g"], rec)
    de = deta.cpu().numpy()
    say(f"  J gpu={J:.12e} oracle={Jo:.12e}")
    assert abs(J - Jo) <= 1e-9 * Jo
    assert np.linalg.norm(db - dbo) <= 1e-6 * np.linalg.norm(dbo)
    assert np.linalg.norm(de - deo) <= 1e-6 * np.linalg.norm(deo)
    model.close()


def test_tet_layout(P):
    """Tetrahedral rows (P1 Kuhn: 15 entries inside, fewer on the walls):
    RCM narrows the random numbering's band and the sorted slices pad less."""
    wl = W.workload(6, elems=(24, 16, 16))
    mesh = wl["mesh"]
    out = {}
    for order, sigma in (("given", 0), ("rcm", 0), ("rcm", 256)):
        m = P.Helmholtz(mesh, wl["beta"], order=order, sigma=sigma)
        lay = m.layout()
        assert np.array_equal(lay["perm"], P.node_order(mesh, order, sigma))
        out[(order, sigma)] = (lay["slots"] / m.sizes()["nnz"], lay["bandwidth"])
        m.close()
    say("  padding, bandwidth:", out)
    assert out[("rcm", 0)][1] < out[("given", 0)][1] / 10
    assert out[("rcm", 256)][0] < out[("given", 0)][0]


def test_schwarz_rejects_tetrahedra(P):
    wl = W.workload(6, elems=(4, 3, 3))
    m = P.Helmholtz(wl["mesh"], wl["beta"])
    m.set_frequency(100.0)
    f = m.load(_t(wl["g"]))
    with pytest.raises(P.HzError):
        m.solve(f, method="schwarz")
    m.close()
