"""GPU parity of the core path against the oracle: operator formation, the
sparse product, load, reductions, FP64 and mixed-precision solves, exact
special cases, and error handling.  Calls go through the C ABI."""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, helmholtz as H, krylov

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2112_00087_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return pkg


def _gpu_model(P, mesh, beta, eta=None):
    return P.Helmholtz(mesh, beta, eta)


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.complex128), device="cuda")


def _np(t):
    return t.detach().cpu().numpy()


MESHES = [(1, 1, 1), (2, 2, 2), (4, 3, 2), (20, 12, 10), (33, 17, 9)]


def _model_in_form(P, mesh, beta, eta, form):
    """A context whose solvers use the given storage form: "stencil" (a box,
    no absorption field), "split" (stencil form switched off by
    HZ_STENCIL=0), "complex" (split form switched off by HZ_SPLIT=0), or
    "eta" (absorption field: every entry complex, complex form)."""
    env = {"HZ_SPLIT": "0" if form == "complex" else "1", "HZ_STENCIL": "1" if form == "stencil" else "0"}
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return _gpu_model(P, mesh, beta, eta)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("form", ["stencil", "split"])
def test_spmv_full_vector_mid_size(P, form):
    """80x48x40 box (162,729 rows: 636 blocks of 256 rows, past the 64
    blocks at which the chunked XCD mapping of blocks to row ranges starts,
    with a tail outside its whole rounds): every row of the product in both
    box forms against the oracle's assembled operator, to the same entrywise
    bound as the small meshes."""
    say("spmv full vector 80x48x40", form)
    wl = W.workload(1, elems=(80, 48, 40))
    mesh = wl["mesh"]
    S = H.System(mesh, wl["beta"], None)
    model = _model_in_form(P, mesh, wl["beta"], None, form)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(mesh["n_nodes"]) + 1j * rng.standard_normal(mesh["n_nodes"])
    for f in (0.0, 250.0):
        A = S.operator(W.wavenumber(f))
        model.set_frequency(f)
        y = _np(model.apply(_t(x)))
        yref = A @ x
        bound = 1e-14 * (abs(A) @ np.abs(x)) + 1e-300
        bad = np.flatnonzero(np.abs(y - yref) > bound)
        assert bad.size == 0, (f, bad[:10], np.max(np.abs(y - yref) / bound))
    model.close()


@pytest.mark.parametrize("form", ["eta", "split", "stencil", "complex"])
@pytest.mark.parametrize("elems", MESHES)
def test_spmv_diag_load_parity(P, elems, form):
    say("spmv parity", elems, form)
    wl = W.workload(1, elems=elems)
    mesh = wl["mesh"]
    rng = np.random.default_rng(7)
    eta = rng.uniform(0, 0.02, mesh["n_elems"]) if form == "eta" else None
    S = H.System(mesh, wl["beta"], eta)
    model = _model_in_form(P, mesh, wl["beta"], eta, form)
    x = rng.standard_normal(mesh["n_nodes"]) + 1j * rng.standard_normal(mesh["n_nodes"])
    for f in (0.0, 100.0, 250.0):
        k = W.wavenumber(f)
        A = S.operator(k)
        model.set_frequency(f)
        y = _np(model.apply(_t(x)))
        yref = A @ x
        bound = 1e-14 * (abs(A) @ np.abs(x)) + 1e-300
        assert np.all(np.abs(y - yref) <= bound), (f, np.max(np.abs(y - yref) / bound))
        d = _np(model.diag())
        # A_ii sums four assembled terms, each a sum over <= 8 elements x 8 Gauss
        # points formed in a different (equally valid) order by library and oracle:
        # allow 1e-14 of the magnitudes, the same bound as the product above
        mag = (np.abs(S.asm["K"].diagonal()) + k * k * np.abs(S.asm["M"].diagonal())
               + (k * k * np.abs(S.Meta.diagonal()) if S.Meta is not None else 0.0)
               + k * np.abs(S.Bbeta.diagonal()))
        assert np.all(np.abs(d - A.diagonal()) <= 1e-14 * mag)
    g = wl["g"] if np.any(wl["g"]) else rng.standard_normal(mesh["n_nodes"]) + 0j
    f = _np(model.load(_t(g)))
    fref = S.load(g)
    assert np.allclose(f, fref, rtol=1e-14, atol=1e-16 * np.abs(fref).max())
    model.close()


def test_dotc_parity_and_determinism(P):
    wl = W.workload(0)
    model = _gpu_model(P, wl["mesh"], wl["beta"])
    rng = np.random.default_rng(3)
    for n in (1, 255, 256, 3003, 1_000_003):
        a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        at, bt = _t(a), _t(b)
        v1 = model.dotc(at, bt)
        v2 = model.dotc(at, bt)
        assert v1 == v2                      # fixed reduction order: bitwise reproducible
        ref = np.vdot(a, b)
        gamma = n * 1.2e-16
        assert abs(v1 - ref) <= 2 * gamma * np.sum(np.abs(a) * np.abs(b)) + 1e-300
    model.close()


@pytest.mark.parametrize("method,kw", [("bicgstab", {}), ("tfqmr", {}), ("bicgstabl", dict(restart=4)),
                                       ("gmres", dict(restart=30))])
def test_solves_are_bitwise_reproducible(P, method, kw):
    """Every reduction has a fixed order (a block's wave sums added in wave
    order by whichever wave finishes last, then the blocks in order), so the
    same solve run twice gives the same iterate and counts bit for bit, on a
    mesh of many blocks (21,525 nodes: 85 blocks of 256 rows).  Converged or
    not within the cap, the two runs must agree."""
    say("bitwise reproducible", method)
    wl = W.workload(1, elems=(40, 24, 20))
    m = _gpu_model(P, wl["mesh"], wl["beta"])
    m.set_frequency(150.0)
    f = m.load(_t(wl["g"]))
    runs = [m.solve(f, method=method, tol=1e-8, max_matvec=4000, **kw) for _ in range(2)]
    (p1, i1), (p2, i2) = runs
    say(f"  {i1}")
    assert np.isfinite(i1["relres_true"])
    assert torch.equal(p1, p2)
    for key in ("status", "iters", "matvecs", "relres_true"):
        assert i1[key] == i2[key], (key, i1, i2)
    m.close()


@pytest.fixture(scope="module")
def c0(P):
    wl = W.workload(0)
    S = H.System(wl["mesh"], wl["beta"])
    k = W.wavenumber(wl["freqs"][0])
    A = S.operator(k)
    f = S.load(wl["g"])
    x = direct.SparseLU(A).solve(f)
    model = _gpu_model(P, wl["mesh"], wl["beta"])
    model.set_frequency(wl["freqs"][0])
    yield dict(wl=wl, A=A, f=f, x=x, model=model)
    model.close()


@pytest.mark.parametrize("method,precision", [("gmres", "fp64"), ("bicgstab", "fp64"),
                                              ("gmres", "mixed"), ("bicgstab", "mixed")])
def test_solve_workload0(c0, method, precision):
    say("solve workload 0", method, precision)
    m = c0["model"]
    p, info = m.solve(_t(c0["f"]), method=method, precision=precision, restart=30, tol=1e-8)
    p = _np(p)
    rel = H.relres(c0["A"], p, c0["f"])
    err = np.linalg.norm(p - c0["x"]) / np.linalg.norm(c0["x"])
    say(f"  info={info} oracle relres={rel:.3e} relerr={err:.3e}")
    assert info["status"] == 0
    assert rel <= 1e-8
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel + 1e-15
    assert err <= 1e-6


@pytest.mark.parametrize("form", ["complex", "split"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_other_form_solve_matches_oracle(P, c0, precision, form):
    """The same solve with the stencil (and split) storage forms switched off."""
    wl = c0["wl"]
    m = _model_in_form(P, wl["mesh"], wl["beta"], None, form)
    m.set_frequency(wl["freqs"][0])
    assert m.spmv_bytes("fp64", "solver") == m.spmv_bytes("fp64", form)
    p, info = m.solve(_t(c0["f"]), method="bicgstab", precision=precision, tol=1e-8)
    p = _np(p)
    rel = H.relres(c0["A"], p, c0["f"])
    err = np.linalg.norm(p - c0["x"]) / np.linalg.norm(c0["x"])
    say(f"  {form} form {precision}: info={info} relres={rel:.3e} relerr={err:.3e}")
    assert info["status"] == 0 and rel <= 1e-8 and err <= 1e-6
    m.close()


def test_split_and_stencil_form_bytes(c0):
    """On a box without absorption field the solvers run the stencil form
    (split values at implied neighbour columns); the algorithmic bytes of
    each form follow the documented formulas."""
    m = c0["model"]
    n, nnz = m.sizes()["n_nodes"], m.sizes()["nnz"]
    bs, bc = m.spmv_bytes("fp64", "split"), m.spmv_bytes("fp64", "complex")
    bst = m.spmv_bytes("fp64", "stencil")
    assert bc == 20 * nnz + 4 * (n + 1) + 32 * n
    assert m.spmv_bytes("fp64", "solver") == bst < bs < bc
    assert bs - bst == 2 * nnz                      # the int16 column offsets
    # every wall node's row is in the imaginary list; interior rows two layers
    # in are not: n_imag lies between the wall entries and all entries
    n_imag = (bs - 10 * nnz - 4 * (n + 1) - 32 * n) / 12
    assert n_imag == int(n_imag) and 0 < n_imag < nnz
    assert m.spmv_bytes("mixed", "split") == 6 * nnz + 8 * n_imag + 4 * (n + 1) + 16 * n
    assert m.spmv_bytes("mixed", "stencil") == 4 * nnz + 8 * n_imag + 4 * (n + 1) + 16 * n


@pytest.mark.parametrize("l,precision", [(1, "fp64"), (2, "fp64"), (4, "fp64"), (8, "fp64"), (4, "mixed"),
                                         (8, "mixed")])
def test_bicgstab_l_workload0(c0, l, precision):
    say("bicgstab(l) workload 0", l, precision)
    m = c0["model"]
    p, info = m.solve(_t(c0["f"]), method="bicgstabl", restart=l, precision=precision, tol=1e-8)
    p = _np(p)
    rel = H.relres(c0["A"], p, c0["f"])
    err = np.linalg.norm(p - c0["x"]) / np.linalg.norm(c0["x"])
    say(f"  info={info} oracle relres={rel:.3e} relerr={err:.3e}")
    assert info["status"] == 0 and rel <= 1e-8 and err <= 1e-6
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel + 1e-15
    if precision == "fp64":
        ref = krylov.bicgstab_l(c0["A"], c0["f"], l=l, tol=1e-8)
        say(f"  cycles gpu {info['iters']} oracle {ref.iters}")
        # Gram-matrix (GPU) and Gram-Schmidt (oracle) minimal-residual steps
        # agree in exact arithmetic: the cycle counts stay close
        assert abs(info["iters"] - ref.iters) <= max(5, 0.25 * ref.iters)
        # the remaining products are true residuals: the start and the check at the end
        assert 2 <= info["matvecs"] - 2 * l * info["iters"] <= 10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tfqmr_workload0(c0, precision):
    say("tfqmr workload 0", precision)
    m = c0["model"]
    p, info = m.solve(_t(c0["f"]), method="tfqmr", precision=precision, tol=1e-8)
    p = _np(p)
    rel = H.relres(c0["A"], p, c0["f"])
    err = np.linalg.norm(p - c0["x"]) / np.linalg.norm(c0["x"])
    say(f"  info={info} oracle relres={rel:.3e} relerr={err:.3e}")
    assert info["status"] == 0 and rel <= 1e-8 and err <= 1e-6
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel + 1e-15
    if precision == "fp64":
        ref = krylov.tfqmr(c0["A"], c0["f"], tol=1e-8)
        say(f"  half-steps gpu {info['iters']} oracle {ref.iters}")
        assert abs(info["iters"] - ref.iters) <= max(10, 0.2 * ref.iters)


def test_bicgstab_l_rejects_bad_l(c0):
    import paper_2112_00087_amd as P
    for l in (0, 9):
        with pytest.raises(P.HzError):
            c0["model"].solve(_t(c0["f"]), method="bicgstabl", restart=l)


def test_gpu_gmres_matches_oracle_iteration_count_roughly(c0):
    m = c0["model"]
    _, info = m.solve(_t(c0["f"]), method="gmres", restart=30, tol=1e-8)
    ref = krylov.gmres(c0["A"], c0["f"], m=30, tol=1e-8)
    say("gmres iters gpu", info["iters"], "oracle", ref.iters)
    # CGS2 vs MGS: iteration counts agree to within a few steps per restart
    assert abs(info["iters"] - ref.iters) <= max(10, 0.1 * ref.iters)


def test_p4_exact_one_d_on_gpu(P):
    from test_oracle_fem import _one_d_exact
    nx, ny, nz = 12, 3, 2
    mesh = W.box_mesh(nx, ny, nz)
    beta = np.zeros(6, complex)
    beta[1] = 0.3 + 0.1j
    S = H.System(mesh, beta)
    g0 = 0.7 - 0.4j
    f = S.asm["B0"][0] @ np.full(mesh["n_nodes"], g0)
    model = _gpu_model(P, mesh, beta)
    model.set_frequency(120.0)
    for method in ("gmres", "bicgstab"):
        p, info = model.solve(_t(f), method=method, tol=1e-13, restart=60)
        exact = _one_d_exact(nx, 1.8 / nx, W.wavenumber(120.0), g0, beta[1])
        i = np.arange(mesh["n_nodes"]) % (nx + 1)
        assert np.abs(_np(p) - exact[i]).max() <= 1e-10 * np.abs(exact).max(), info
    model.close()


def test_p9_real_case_gives_zero_imaginary_part(P):
    mesh = W.box_mesh(6, 4, 3)
    model = _gpu_model(P, mesh, np.zeros(6))
    model.set_frequency(111.0)
    rng = np.random.default_rng(9)
    f = rng.standard_normal(mesh["n_nodes"]) + 0j
    for method in ("gmres", "bicgstab"):
        p, info = model.solve(_t(f), method=method, tol=1e-10)
        assert info["status"] == 0
        assert np.abs(_np(p).imag).max() == 0.0
    model.close()


def test_error_contract_on_gpu(P):
    wl = W.workload(0)
    model = _gpu_model(P, wl["mesh"], wl["beta"])
    f = _t(np.ones(model.n))
    with pytest.raises(P.HzError) as e:
        model.solve(f)
    assert e.value.code == P.HZ_ERR_STATE
    model.set_frequency(100.0)
    bad = f.clone()
    bad[5] = complex(np.nan, 0)
    with pytest.raises(P.HzError) as e:
        model.solve(bad)
    assert e.value.code == P.HZ_ERR_INVALID
    p, info = model.solve(f, max_matvec=3)
    assert info["status"] == P.HZ_NOT_CONVERGED and info["matvecs"] <= 4
    p, info = model.solve(f, method="bicgstab", max_matvec=3)
    assert info["status"] == P.HZ_NOT_CONVERGED
    z, info = model.solve(torch.zeros_like(f))
    assert info["status"] == 0 and torch.count_nonzero(z) == 0
    with pytest.raises(P.HzError):
        model.solve(f, restart=0)
    model.set_params(beta=wl["beta"])
    with pytest.raises(P.HzError) as e:
        model.solve(f)
    assert e.value.code == P.HZ_ERR_STATE
    model.close()


def test_initial_guess_is_used(c0):
    m = c0["model"]
    p, info = m.solve(_t(c0["f"]), x0=_t(c0["x"]), method="bicgstab", tol=1e-8)
    assert info["status"] == 0 and info["matvecs"] <= 3
