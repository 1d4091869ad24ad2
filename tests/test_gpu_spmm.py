"""The frequency sweep's multi-vector product (hz_apply_sweep) column by
column against the oracle's assembled operator, in the autotuner's pick
and in every forced product variant (row-wise gathering and stencil
form), in FP64 and in the complex64 form of the mixed sweep.

Bound, per output entry i and column c with k = k_c (Sec. 4, the product
of the discretised operator): the FP64 product sums at most 27 stiffness,
mass and absorption terms plus the boundary terms, each rounded a few
times, so |y_i - y_ref,i| <= 1e-13 B_i with
B_i = sum_j (|K_ij| + |m(k)| |M_ij| + k |(B beta)_ij| + k^2 |Meta_ij|) |x_j|, m(k) = k^2 or,
with Galerkin least-squares stabilisation, k^2 (1 - tau k^2)
(about 450 unit roundoffs, far below the O(B_i / 27) error of one
misplaced entry).  The complex64 product rounds x and the operator to
24-bit mantissas and forms the stiffness in difference form
K_ij (x_j - x_i): |y_i - y_ref,i| <= 1e-5 (B_i + |x_i| sum_j |K_ij|).
"""
import functools
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
def P():
    import paper_2112_00087_amd as pkg
    assert torch.cuda.is_available()
    return pkg


# stencil-form variant codes: 1, the pairs' broadcast (0 readlane, 1 LDS),
# blocks of pw x ph lines, four digits of z chunks
def zl_code(pw, ph, nzc, bc=0):
    return 10000000 + bc * 1000000 + pw * 100000 + ph * 10000 + nzc


ZL_FORCED = [zl_code(1, 1, 1), zl_code(2, 1, 3), zl_code(2, 2, 2), zl_code(4, 2, 16),
             zl_code(1, 1, 2, 1), zl_code(2, 1, 5, 1), zl_code(4, 2, 8, 1)]
ROWWISE = [11256, 2128]   # one lane per column / 256 threads / XCD rows; two per lane / 128 threads


def _cases():
    # (workload, mesh size, Galerkin least-squares mass coefficient)
    return {"box": (2, (20, 12, 10), False), "box-eta": (4, (14, 9, 8), False), "kuhn": (5, (6, 4, 4), False),
            "box-gls": (2, (16, 10, 8), True), "tet": (6, (6, 4, 4), False)}


@functools.lru_cache(maxsize=None)
def _system(name):
    cfg, elems, gls = _cases()[name]
    wl = W.workload(cfg, elems=elems)
    S = H.System(wl["mesh"], wl["beta"], wl["eta"], gls=gls)
    return wl, S


def _model(P, name):
    wl, S = _system(name)
    return P.Helmholtz(wl["mesh"], wl["beta"], wl["eta"], gls=_cases()[name][2])


@functools.lru_cache(maxsize=None)
def _reference(name, nfreq):
    wl, S = _system(name)
    freqs = np.linspace(20, 300, 64)[:: max(1, 64 // nfreq)][:nfreq]
    rng = np.random.default_rng(100 + nfreq)
    X = rng.standard_normal((S.n, nfreq)) + 1j * rng.standard_normal((S.n, nfreq))
    K, M = S.asm["K"], S.asm["M"]
    aK, aM, aB = abs(K), abs(M), abs(S.Bbeta)
    aE = None if S.Meta is None else abs(S.Meta)
    Y = np.empty_like(X)
    B = np.empty(X.shape)
    Bd = np.empty(X.shape)
    ksum = np.asarray(aK.sum(axis=1)).ravel()
    for c, f in enumerate(freqs):
        k = W.wavenumber(f)
        Y[:, c] = S.operator(k) @ X[:, c]
        ax = np.abs(X[:, c])
        m = S.mass_coefficient(k)   # k^2, or k^2 (1 - tau k^2) with GLS
        B[:, c] = aK @ ax + abs(m) * (aM @ ax) + k * (aB @ ax) + (0.0 if aE is None else k * k * (aE @ ax))
        Bd[:, c] = B[:, c] + ax * ksum
    return freqs, X, Y, B, Bd


def _check(name, nfreq, precision, Yg):
    freqs, X, Y, B, Bd = _reference(name, nfreq)
    err = np.abs(Yg - Y)
    bound = 1e-13 * B if precision == "fp64" else 1e-5 * Bd
    worst = np.max(err / np.maximum(bound, 1e-300))
    say(f"  {name} nfreq={nfreq} {precision}: worst err/bound {worst:.3g}")
    assert np.all(err <= bound), (name, nfreq, precision, worst)


def _fits(code, nfreq, precision, name):
    """Whether a forced variant applies at this width (the library falls back
    to its autotuner otherwise)."""
    s = 1 << int(np.ceil(np.log2(nfreq))) if nfreq > 1 else 1
    if code < 10000000:
        return True
    if name in ("kuhn", "tet"):
        return False   # no stencil form off a box
    bc = code // 1000000 % 10
    return s == 64 or (s == 32 and bc == 1)   # 32 columns: two lines per wave, pairs through LDS


@pytest.mark.parametrize("name", ["box", "box-eta", "kuhn", "box-gls", "tet"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nfreq", [64, 33, 20, 8, 4, 1])
def test_apply_sweep_autotuned(P, name, precision, nfreq):
    say("apply_sweep autotuned", name, precision, nfreq)
    freqs, X, _, _, _ = _reference(name, nfreq)
    model = _model(P, name)
    Yg, v = model.apply_sweep(freqs, X, precision=precision)
    say("  variant", v)
    _check(name, nfreq, precision, Yg.cpu().numpy())
    model.close()


@pytest.mark.parametrize("code", ZL_FORCED + ROWWISE)
@pytest.mark.parametrize("name", ["box", "box-eta", "kuhn", "box-gls", "tet"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_sweep_forced_variant(P, code, name, precision, monkeypatch):
    monkeypatch.setenv("HZ_SPMM_VARIANT", str(code))
    model = _model(P, name)
    for nfreq in (64, 33, 20, 16, 5):
        say("apply_sweep forced", code, name, precision, nfreq)
        freqs, X, _, _, _ = _reference(name, nfreq)
        Yg, v = model.apply_sweep(freqs, X, precision=precision)
        if _fits(code, nfreq, precision, name):
            assert v == code, (v, code)
        _check(name, nfreq, precision, Yg.cpu().numpy())
    model.close()


def test_apply_sweep_rejects_bad_arguments(P):
    wl, S = _system("box")
    model = P.Helmholtz(wl["mesh"], wl["beta"])
    X = torch.zeros((S.n, 65), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.HzError):
        model.apply_sweep(np.linspace(20, 300, 65), X)
    X = torch.zeros((S.n, 2), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.HzError):
        model.apply_sweep(np.array([100.0, np.nan]), X)
    model.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_sweep_full_size_sampled_rows(P, precision):
    """The 80x48x40 box with its 64 sweep frequencies (the product the bench
    times): 3000 sampled rows of every column against the oracle's rows of
    A(k_c), built from the elements and faces that touch them."""
    say("apply_sweep full size", precision)
    wl = W.workload(2)
    mesh = wl["mesh"]
    freqs = wl["freqs"]
    n = mesh["n_nodes"]
    rng = np.random.default_rng(7)
    X = rng.standard_normal((n, freqs.size)) + 1j * rng.standard_normal((n, freqs.size))
    model = P.Helmholtz(mesh, wl["beta"])
    Yg, v = model.apply_sweep(freqs, X, precision=precision)
    say("  variant", v)
    Yg = Yg.cpu().numpy()
    model.close()
    rows = np.sort(rng.choice(n, size=3000, replace=False))
    zero = np.zeros(6, dtype=np.complex128)
    Kr = H.rows_of_operator(mesh, 0.0, zero, None, rows).real
    Mr = Kr - H.rows_of_operator(mesh, 1.0, zero, None, rows).real
    aK, aM = abs(Kr), abs(Mr)
    ksum = np.asarray(aK.sum(axis=1)).ravel()
    worst = 0.0
    for c, f in enumerate(freqs):
        k = W.wavenumber(f)
        Ar = H.rows_of_operator(mesh, k, wl["beta"], None, rows)
        aB = abs(Ar - H.rows_of_operator(mesh, k, zero, None, rows))
        ax = np.abs(X[:, c])
        B = aK @ ax + k * k * (aM @ ax) + aB @ ax
        if precision == "mixed":
            B = B + ax[rows] * ksum
        err = np.abs(Yg[rows, c] - Ar @ X[:, c])
        bound = (1e-13 if precision == "fp64" else 1e-5) * B
        worst = max(worst, float(np.max(err / bound)))
        assert np.all(err <= bound), (c, f, float(np.max(err / bound)))
    say(f"  worst err/bound {worst:.3g}")
