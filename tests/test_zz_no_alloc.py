"""The allocation-free dot product (hz_dotc_noalloc) against hz_dotc,
called through the C ABI: bitwise equal results on two calls in a row, the
second with a smaller input, and the library's device memory unchanged."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_dotc_noalloc_matches_dotc_twice():
    from paper_2112_00087_amd import Helmholtz, hz
    assert torch.cuda.is_available()
    L = hz.lib()
    wl = W.workload(0)
    model = Helmholtz(wl["mesh"], wl["beta"])
    rng = np.random.default_rng(7)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    for n in (3 * 1024 * 1024 + 77, 4099):     # second call smaller; both ragged
        say(f"noalloc dot n={n}")
        a = torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n), device="cuda")
        b = torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n), device="cuda")
        torch.cuda.synchronize()
        ref = hz.hz_c128()
        hz.check(L.hz_dotc(model.ctx, n, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.byref(ref)), False)
        before = model.sizes()["device_bytes"]
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        hz.check(L.hz_dotc_noalloc(model.ctx, n, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                   C.c_void_p(out.data_ptr())), False)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        got = out.cpu().numpy()
        say(f"  dotc {ref.re!r} {ref.im!r}  noalloc {got[0]!r} {got[1]!r}")
        assert got[0] == ref.re and got[1] == ref.im
        # and both agree with the exact sum within the dot-product bound
        an, bn = a.cpu().numpy(), b.cpu().numpy()
        exact = np.vdot(an, bn)
        bound = 2 * n * 1.2e-16 * np.sum(np.abs(an) * np.abs(bn))
        assert abs(complex(got[0], got[1]) - exact) <= bound
        assert model.sizes()["device_bytes"] == before
    # invalid arguments are rejected without touching the output
    assert L.hz_dotc_noalloc(model.ctx, -1, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                             C.c_void_p(out.data_ptr())) == hz.HZ_ERR_INVALID
    assert L.hz_dotc_noalloc(model.ctx, 4, None, C.c_void_p(b.data_ptr()),
                             C.c_void_p(out.data_ptr())) == hz.HZ_ERR_INVALID
    model.close()
