"""GPU Schwarz decomposition (batched subdomain solves + interface GMRES)
against the oracle: the global solution, the trivial partition, and the
iterate of the plain Schwarz iteration."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import direct, helmholtz as H, schwarz

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2112_00087_amd as pkg
    assert torch.cuda.is_available()
    return pkg


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.complex128), device="cuda")


def _case(elems, freq, eta=False, seed=2):
    wl = W.workload(3, elems=elems)
    mesh = wl["mesh"]
    rng = np.random.default_rng(seed)
    et = rng.uniform(0, 0.02, mesh["n_elems"]) if eta else None
    S = H.System(mesh, wl["beta"], et)
    k = W.wavenumber(freq)
    A = S.operator(k)
    f = S.load(wl["g"])
    return wl, mesh, et, k, A, f


@pytest.mark.parametrize("parts,inner,eta", [((2, 2, 1), "bicgstab", False), ((2, 2, 2), "gmres", True),
                                             ((3, 1, 2), "bicgstab", True), ((2, 1, 2), "bicgstabl", False)])
def test_schwarz_fp64_matches_global_solution(P, parts, inner, eta):
    say("schwarz fp64", parts, inner, eta)
    wl, mesh, et, k, A, f = _case((12, 8, 6), 150.0, eta)
    model = P.Helmholtz(mesh, wl["beta"], et, parts=parts)
    model.set_frequency(150.0)
    p, info = model.solve(_t(f), method="schwarz", restart=40, tol=1e-9, inner_tol=1e-12,
                          dd_inner=inner, inner_restart=4 if inner == "bicgstabl" else 30, max_matvec=5000)
    say("  ", info)
    p = p.cpu().numpy()
    x = direct.SparseLU(A).solve(f)
    rel = H.relres(A, p, f)
    assert info["status"] == 0 and rel <= 1e-9 * 1.01
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel
    assert np.linalg.norm(p - x) <= 1e-6 * np.linalg.norm(x)
    model.close()


def test_schwarz_trivial_partition_is_global_solve(P):
    wl, mesh, et, k, A, f = _case((8, 6, 4), 120.0)
    model = P.Helmholtz(mesh, wl["beta"], parts=(1, 1, 1))
    model.set_frequency(120.0)
    p, info = model.solve(_t(f), method="schwarz", tol=1e-10, inner_tol=1e-12, dd_inner="bicgstab")
    assert info["status"] == 0 and info["iters"] == 0
    x = direct.SparseLU(A).solve(f)
    assert np.linalg.norm(p.cpu().numpy() - x) <= 1e-9 * np.linalg.norm(x)
    model.close()


@pytest.mark.parametrize("alpha_of_k", [lambda k: 1j * k, lambda k: 0.5 * k + 1.5j * k,
                                        lambda k: (0.5 * k + 1.5j * k, 3.0 * k + 0.2j * k)],
                         ids=["ik", "general", "two-sided"])
def test_schwarz_plain_iteration_matches_oracle_history(P, alpha_of_k):
    wl, mesh, et, k, A, f = _case((8, 6, 4), 90.0)
    parts = (2, 2, 1)
    alpha = alpha_of_k(k)
    D = schwarz.Schwarz(mesh, parts, wl["beta"], None, k, f, alpha=alpha)
    model = P.Helmholtz(mesh, wl["beta"], parts=parts)
    model.set_frequency(90.0)
    for n_it in (1, 4, 10):
        a_lo, a_hi = alpha if isinstance(alpha, tuple) else (alpha, 0j)
        p, info = model.solve(_t(f), method="schwarz", tol=1e-12, inner_tol=1e-13, dd_inner="gmres",
                              inner_restart=60, dd_richardson=n_it, dd_alpha=a_lo, dd_alpha2=a_hi)
        u, lams, hist = D.richardson(n_it + 1, A, f)
        err = np.linalg.norm(p.cpu().numpy() - u) / np.linalg.norm(u)
        say(f"  plain Schwarz {n_it}: rel diff {err:.2e}, oracle relres {hist[-1, 1]:.3e}, gpu {info['relres_true']:.3e}")
        assert err <= 1e-8
        assert abs(info["relres_true"] - hist[-1, 1]) <= 1e-6 * hist[-1, 1]
    model.close()


def test_schwarz_mixed_local_solves(P):
    wl, mesh, et, k, A, f = _case((20, 12, 10), 150.0)
    model = P.Helmholtz(mesh, wl["beta"], parts=(2, 2, 2))
    model.set_frequency(150.0)
    p, info = model.solve(_t(f), method="schwarz", precision="mixed", tol=1e-8, inner_tol=1e-10,
                          dd_inner="bicgstab", restart=40, max_matvec=5000)
    say("  mixed schwarz", info)
    rel = H.relres(A, p.cpu().numpy(), f)
    x = direct.SparseLU(A).solve(f)
    assert info["status"] == 0 and rel <= 1e-8 * 1.01
    assert np.linalg.norm(p.cpu().numpy() - x) <= 1e-6 * np.linalg.norm(x)
    model.close()


def test_schwarz_rejects_unstructured_or_bad_parts(P):
    wl, mesh, et, k, A, f = _case((4, 3, 2), 100.0)
    bad = dict(mesh, elems=(0, 0, 0))
    model = P.Helmholtz(bad, wl["beta"], parts=(2, 1, 1))
    model.set_frequency(100.0)
    with pytest.raises(P.HzError):
        model.solve(_t(f), method="schwarz")
    model.close()
    model = P.Helmholtz(mesh, wl["beta"], parts=(9, 1, 1))
    model.set_frequency(100.0)
    with pytest.raises(P.HzError):
        model.solve(_t(f), method="schwarz")
    model.close()


def _pair(P, k, mesh, parts):
    """The optimised two-sided coefficients for a partition (smallest
    subdomain width, smallest mesh spacing), as the library's default."""
    nx, ny, nz = mesh["elems"]
    sp = [1.8 / nx, 1.2 / ny, 1.0 / nz]
    H_sub = min(sp[d] * (mesh["elems"][d] // parts[d]) for d in range(3))
    return P.dd_alpha(k, H_sub, min(sp), sides=2)


@pytest.mark.parametrize("precision,itol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_schwarz_4x3x2_partition_matches_global_solution(P, precision, itol):
    """The configured partition, 4 x 3 x 2 = 24 subdomains (interior parts
    with 5 face neighbours, cross points where 8 subdomains meet), on a
    40x24x20 box (subdomains of 10x8x10 elements) at 150 Hz: interface GMRES
    with the optimised two-sided coefficients and BiCGStab(4) local solves,
    complex128 or complex64 with FP64 refinement, against the oracle's direct
    solution of the global system."""
    say("schwarz 4x3x2", precision)
    wl, mesh, et, k, A, f = _case((40, 24, 20), 150.0)
    model = P.Helmholtz(mesh, wl["beta"], parts=(4, 3, 2))
    model.set_frequency(150.0)
    p, info = model.solve(_t(f), method="schwarz", restart=300, tol=1e-8, inner_tol=itol, precision=precision,
                          dd_inner="bicgstabl", inner_restart=4, max_matvec=300)
    say("  ", info)
    p = p.cpu().numpy()
    x = direct.SparseLU(A).solve(f)
    rel = H.relres(A, p, f)
    err = np.linalg.norm(p - x) / np.linalg.norm(x)
    say(f"  oracle relres {rel:.3e}, relerr vs direct {err:.3e}")
    assert info["status"] == 0 and rel <= 1e-8 * 1.01
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel
    assert err <= 1e-6
    model.close()


def test_schwarz_4x3x2_plain_iteration_matches_oracle_history(P):
    """Plain Schwarz iterations on the 4 x 3 x 2 partition (20x12x10 box,
    subdomains of 5x4x5 elements) with the optimised two-sided pair: the GPU
    iterate equals the oracle's (direct local solves) after 1, 4 and 10
    iterations, and so do the global residuals."""
    wl, mesh, et, k, A, f = _case((20, 12, 10), 150.0)
    parts = (4, 3, 2)
    a_lo, a_hi = _pair(P, k, mesh, parts)
    say(f"  pair {a_lo:.4g} {a_hi:.4g}")
    D = schwarz.Schwarz(mesh, parts, wl["beta"], None, k, f, alpha=(a_lo, a_hi))
    model = P.Helmholtz(mesh, wl["beta"], parts=parts)
    model.set_frequency(150.0)
    for n_it in (1, 4, 10):
        p, info = model.solve(_t(f), method="schwarz", tol=1e-12, inner_tol=1e-13, dd_inner="gmres",
                              inner_restart=60, dd_richardson=n_it, dd_alpha=a_lo, dd_alpha2=a_hi)
        u, lams, hist = D.richardson(n_it + 1, A, f)
        err = np.linalg.norm(p.cpu().numpy() - u) / np.linalg.norm(u)
        say(f"  plain Schwarz {n_it}: rel diff {err:.2e}, oracle relres {hist[-1, 1]:.3e}, gpu {info['relres_true']:.3e}")
        assert err <= 1e-8
        assert abs(info["relres_true"] - hist[-1, 1]) <= 1e-6 * hist[-1, 1]
    model.close()
