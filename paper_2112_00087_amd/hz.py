"""ctypes binding of ``libhz.so`` (C ABI in ``include/hz.h``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device vectors are torch tensors (complex128 / float64, contiguous,
on the library's GPU); torch provides the memory and the stream, nothing else.
If the library is not built, or no GPU is present, calls fail loudly; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhz.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "hz.h")

HZ_OK, HZ_NOT_CONVERGED, HZ_BREAKDOWN = 0, 1, 2
HZ_ERR_INVALID, HZ_ERR_HIP, HZ_ERR_OOM, HZ_ERR_STATE = -1, -2, -3, -4
HZ_GMRES, HZ_BICGSTAB, HZ_SCHWARZ, HZ_BICGSTABL, HZ_TFQMR = 0, 1, 2, 3, 4
HZ_FP64, HZ_MIXED = 0, 1
HZ_JACOBI, HZ_NONE = 0, 1

METHODS = {"gmres": HZ_GMRES, "bicgstab": HZ_BICGSTAB, "schwarz": HZ_SCHWARZ, "bicgstabl": HZ_BICGSTABL, "tfqmr": HZ_TFQMR}
PRECISIONS = {"fp64": HZ_FP64, "mixed": HZ_MIXED}
SPMV_FORMS = {"solver": 0, "complex": 1, "split": 2, "stencil": 3}
ORDERS = {"given": 0, "rcm": 1}
HZ_HEX8, HZ_TET4 = 0, 1


def _connectivity(mesh):
    """Element array and element type of a mesh dict: ``tet`` (4 nodes per
    element) or ``hex`` (8)."""
    if "tet" in mesh:
        return np.ascontiguousarray(mesh["tet"], dtype=np.int32), HZ_TET4
    return np.ascontiguousarray(mesh["hex"], dtype=np.int32), HZ_HEX8


class hz_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class hz_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("n_bfaces", C.c_int32),
                ("xyz", C.POINTER(C.c_double)), ("hex", C.POINTER(C.c_int32)),
                ("bface", C.POINTER(C.c_int32)), ("bface_tag", C.POINTER(C.c_int32)),
                ("bface_src", C.POINTER(C.c_uint8)), ("c", C.c_double), ("rho", C.c_double),
                ("elems", C.c_int32 * 3), ("parts", C.c_int32 * 3), ("order", C.c_int32),
                ("sigma", C.c_int32), ("elem_type", C.c_int32), ("src_kind", C.c_int32),
                ("fe_scheme", C.c_int32)]


class hz_solve_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart", C.c_int32), ("max_matvec", C.c_int32),
                ("precision", C.c_int32), ("precond", C.c_int32), ("inner_restart", C.c_int32),
                ("tol", C.c_double), ("inner_tol", C.c_double), ("dd_alpha", hz_c128),
                ("dd_inner", C.c_int32), ("dd_richardson", C.c_int32), ("dd_alpha2", hz_c128)]


class hz_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("matvecs", C.c_int32),
                ("inner_matvecs", C.c_int32), ("relres_true", C.c_double),
                ("relres_est", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hz error {code}: {msg}")
        self.code = code


_lib = None
VP = C.c_void_p


def header_symbols():
    """Names of the functions declared in include/hz.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hz_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Load libhz.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2112_00087_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    sig = {
        "hz_assemble": (C.c_int, [P(hz_mesh), P(hz_c128), P(C.c_double), VP, P(VP)]),
        "hz_set_params": (C.c_int, [VP, P(hz_c128), P(C.c_double)]),
        "hz_set_frequency": (C.c_int, [VP, C.c_double]),
        "hz_apply": (C.c_int, [VP, VP, VP]),
        "hz_get_diag": (C.c_int, [VP, VP]),
        "hz_load": (C.c_int, [VP, VP, VP]),
        "hz_dotc": (C.c_int, [VP, C.c_int64, VP, VP, P(hz_c128)]),
        "hz_dotc_noalloc": (C.c_int, [VP, C.c_int64, VP, VP, VP]),
        "hz_solve": (C.c_int, [VP, P(hz_solve_opts), VP, VP, P(hz_solve_info)]),
        "hz_solve_sweep": (C.c_int, [VP, C.c_int32, P(C.c_double), VP, VP, P(hz_solve_opts),
                                     P(hz_solve_info)]),
        "hz_solve_adjoint": (C.c_int, [VP, P(hz_solve_opts), VP, VP, VP, P(C.c_double), VP,
                                       P(hz_solve_info)]),
        "hz_time_spmv": (C.c_int, [VP, C.c_int32, C.c_int32, C.c_int32, P(C.c_double)]),
        "hz_spmv_bytes": (C.c_int, [VP, C.c_int32, C.c_int32, P(C.c_int64)]),
        "hz_time_spmm": (C.c_int, [VP, C.c_int32, P(C.c_double), C.c_int32, C.c_int32, P(C.c_double),
                                   P(C.c_int64), P(C.c_int32)]),
        "hz_apply_sweep": (C.c_int, [VP, C.c_int32, P(C.c_double), C.c_int32, VP, VP, P(C.c_int32)]),
        "hz_dd_alpha": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int32, P(hz_c128)]),
        "hz_receiver_energy": (C.c_int, [VP, C.c_int32, P(C.c_int32), VP, P(C.c_double), VP]),
        "hz_node_order": (C.c_int, [P(hz_mesh), P(C.c_int32)]),
        "hz_layout": (C.c_int, [VP, P(C.c_int32), P(C.c_int64), P(C.c_int64), P(C.c_int64)]),
        "hz_sizes": (C.c_int, [VP, P(C.c_int64), P(C.c_int64), P(C.c_int64), P(C.c_int64)]),
        "hz_destroy": (None, [VP]),
        "hz_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error():
    return lib().hz_last_error().decode()


def check(code, allow_positive=True):
    if code < 0 or (code > 0 and not allow_positive):
        raise HzError(code, last_error())
    return code


def make_opts(method="gmres", restart=30, max_matvec=20000, precision="fp64", precond="jacobi",
              tol=1e-8, inner_tol=1e-4, inner_restart=30, dd_alpha=0j, dd_alpha2=0j, dd_inner="gmres",
              dd_richardson=0):
    o = hz_solve_opts()
    o.method = METHODS[method] if isinstance(method, str) else int(method)
    o.restart = restart
    o.max_matvec = max_matvec
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.precond = {"jacobi": HZ_JACOBI, "none": HZ_NONE}[precond] if isinstance(precond, str) else int(precond)
    o.inner_restart = inner_restart
    o.tol = tol
    o.inner_tol = inner_tol
    o.dd_alpha = hz_c128(complex(dd_alpha).real, complex(dd_alpha).imag)
    o.dd_alpha2 = hz_c128(complex(dd_alpha2).real, complex(dd_alpha2).imag)
    o.dd_inner = METHODS[dd_inner] if isinstance(dd_inner, str) else int(dd_inner)
    o.dd_richardson = int(dd_richardson)
    return o


def dd_alpha(k, H, h, sides=2):
    """Optimised Robin coefficients (host computation, hz_dd_alpha): one
    pair of complex numbers (equal for sides=1)."""
    out = (hz_c128 * 2)()
    check(lib().hz_dd_alpha(float(k), float(H), float(h), int(sides), out), False)
    return complex(out[0].re, out[0].im), complex(out[1].re, out[1].im)


def node_order(mesh, order="rcm", sigma=0):
    """Internal numbering hz_assemble would use (host computation,
    hz_node_order): ``perm[p]`` = mesh node of internal row p."""
    hexes, et = _connectivity(mesh)
    m = hz_mesh()
    m.n_nodes = int(np.asarray(mesh["xyz"]).shape[0])
    m.n_elems = hexes.shape[0]
    m.hex = _np_ptr(hexes, C.c_int32)
    m.elem_type = et
    m.order = ORDERS[order] if isinstance(order, str) else int(order)
    m.sigma = int(sigma)
    perm = np.empty(m.n_nodes, dtype=np.int32)
    check(lib().hz_node_order(C.byref(m), _np_ptr(perm, C.c_int32)), False)
    return perm


def _np_ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _beta_array(beta):
    b = np.asarray(beta, dtype=np.complex128).reshape(6)
    arr = (hz_c128 * 6)()
    for w in range(6):
        arr[w] = hz_c128(b[w].real, b[w].imag)
    return arr


def _dev(t, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


class Helmholtz:
    """One assembled mesh on the GPU (wraps an ``hz_ctx``)."""

    def __init__(self, mesh, beta, eta=None, c=340.0, rho=1.2, parts=None, order="given", sigma=0,
                 dirichlet=False, gls=False):
        """``order`` "given" or "rcm" and ``sigma`` (0 or a multiple of 64)
        choose the internal row numbering; vectors stay in the mesh's node
        order either way.  ``dirichlet``: the source faces' nodes carry a
        prescribed pressure (load needs a frequency); ``gls``: Galerkin
        least-squares stabilisation."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Helmholtz needs a ROCm GPU (torch.cuda.is_available() is False)")
        L = lib()
        conn, et = _connectivity(mesh)
        self._keep = dict(
            xyz=np.ascontiguousarray(mesh["xyz"], dtype=np.float64),
            hex=conn,
            bface=np.ascontiguousarray(mesh["bface"], dtype=np.int32),
            tag=np.ascontiguousarray(mesh["bface_tag"], dtype=np.int32),
            src=np.ascontiguousarray(mesh["bface_src"], dtype=np.uint8),
        )
        k = self._keep
        m = hz_mesh()
        m.n_nodes = k["xyz"].shape[0]
        m.n_elems = k["hex"].shape[0]
        m.n_bfaces = k["bface"].shape[0]
        m.xyz = _np_ptr(k["xyz"], C.c_double)
        m.hex = _np_ptr(k["hex"], C.c_int32)
        m.bface = _np_ptr(k["bface"], C.c_int32)
        m.bface_tag = _np_ptr(k["tag"], C.c_int32)
        m.bface_src = _np_ptr(k["src"], C.c_uint8)
        m.c, m.rho = c, rho
        el = mesh.get("elems", (0, 0, 0))
        pa = parts if parts is not None else (0, 0, 0)
        for d in range(3):
            m.elems[d] = int(el[d])
            m.parts[d] = int(pa[d])
        m.order = ORDERS[order] if isinstance(order, str) else int(order)
        m.sigma = int(sigma)
        m.elem_type = et
        m.src_kind = 1 if dirichlet else 0
        m.fe_scheme = 1 if gls else 0
        self.n = m.n_nodes
        self.ne = m.n_elems
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream()
        eta_arr = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        out = C.c_void_p()
        check(L.hz_assemble(C.byref(m), _beta_array(beta),
                            None if eta_arr is None else _np_ptr(eta_arr, C.c_double),
                            C.c_void_p(self.stream.cuda_stream), C.byref(out)), False)
        self.ctx = out
        self.freq = None

    # -------------------------------------------------------------- helpers
    def _vec(self, x=None):
        import torch
        if x is None:
            return torch.zeros(self.n, dtype=torch.complex128, device=self.device)
        return torch.as_tensor(x, dtype=torch.complex128, device=self.device).contiguous()

    def close(self):
        if getattr(self, "ctx", None):
            lib().hz_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        a, b, c_, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().hz_sizes(self.ctx, C.byref(a), C.byref(b), C.byref(c_), C.byref(d)))
        return dict(n_nodes=a.value, n_elems=b.value, nnz=c_.value, device_bytes=d.value)

    def layout(self):
        """Internal numbering (``perm[p]`` = mesh node of internal row p),
        stored sliced-ELL slots, bandwidth and listed imaginary entries."""
        perm = np.empty(self.n, dtype=np.int32)
        sl, bw, ni = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().hz_layout(self.ctx, _np_ptr(perm, C.c_int32), C.byref(sl), C.byref(bw), C.byref(ni)), False)
        return dict(perm=perm, slots=sl.value, bandwidth=bw.value, n_imag=ni.value)

    def time_spmv(self, reps=100, precision="fp64", form="solver"):
        """Average duration (ms) of one sparse product of the given storage form
        ("solver", "complex", "split" or "stencil"), HIP events on the context
        stream."""
        ms = C.c_double()
        check(lib().hz_time_spmv(self.ctx, int(reps), PRECISIONS[precision], SPMV_FORMS[form], C.byref(ms)),
              False)
        return ms.value

    def time_spmm(self, freqs, reps=50, precision="fp64"):
        """(average ms, algorithmic bytes, variant code) of the sweep's
        multi-vector product for these frequencies (hz_time_spmm)."""
        f = np.ascontiguousarray(freqs, dtype=np.float64)
        ms, b, v = C.c_double(), C.c_int64(), C.c_int32()
        check(lib().hz_time_spmm(self.ctx, f.size, _np_ptr(f, C.c_double), PRECISIONS[precision], int(reps),
                                 C.byref(ms), C.byref(b), C.byref(v)), False)
        return ms.value, b.value, v.value

    def spmv_bytes(self, precision="fp64", form="solver"):
        """Algorithmic bytes of one sparse product of the given form."""
        b = C.c_int64()
        check(lib().hz_spmv_bytes(self.ctx, PRECISIONS[precision], SPMV_FORMS[form], C.byref(b)), False)
        return b.value

    # -------------------------------------------------------------- calls
    def set_params(self, beta=None, eta=None):
        b = None if beta is None else _beta_array(beta)
        e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
        check(lib().hz_set_params(self.ctx, b, None if e is None else _np_ptr(e, C.c_double)), False)
        self.freq = None

    def set_frequency(self, freq_hz):
        check(lib().hz_set_frequency(self.ctx, float(freq_hz)), False)
        self.freq = float(freq_hz)

    def apply(self, x, out=None):
        x = self._vec(x)
        y = self._vec() if out is None else out
        check(lib().hz_apply(self.ctx, _dev(x, x.dtype), _dev(y, y.dtype)), False)
        return y

    def diag(self):
        d = self._vec()
        check(lib().hz_get_diag(self.ctx, _dev(d, d.dtype)), False)
        return d

    def load(self, g):
        g = self._vec(g)
        f = self._vec()
        check(lib().hz_load(self.ctx, _dev(g, g.dtype), _dev(f, f.dtype)), False)
        return f

    def dotc(self, a, b):
        import torch
        a = torch.as_tensor(a, dtype=torch.complex128, device=self.device).contiguous()
        b = torch.as_tensor(b, dtype=torch.complex128, device=self.device).contiguous()
        out = hz_c128()
        check(lib().hz_dotc(self.ctx, a.numel(), _dev(a, a.dtype), _dev(b, b.dtype), C.byref(out)), False)
        return complex(out.re, out.im)

    def receiver_energy(self, p, receivers):
        """J = sum_r |p_r|^2 over distinct receiver node ids and its
        derivative g = dJ/dconj(p) (hz_receiver_energy)."""
        p = self._vec(p)
        if hasattr(receivers, "detach"):
            receivers = receivers.detach().cpu().numpy()
        rec = np.ascontiguousarray(np.asarray(receivers, dtype=np.int64).ravel(), dtype=np.int32)
        g = self._vec()
        J = C.c_double(0.0)
        check(lib().hz_receiver_energy(self.ctx, rec.size, _np_ptr(rec, C.c_int32), _dev(p, p.dtype),
                                       C.byref(J), _dev(g, g.dtype)), False)
        return J.value, g

    def solve(self, f, x0=None, **opts):
        f = self._vec(f)
        p = self._vec(x0).clone() if x0 is not None else self._vec()
        info = hz_solve_info()
        code = lib().hz_solve(self.ctx, C.byref(make_opts(**opts)), _dev(f, f.dtype), _dev(p, p.dtype),
                              C.byref(info))
        check(code)
        return p, info.as_dict()

    def solve_sweep(self, freqs, F, P0=None, **opts):
        import torch
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        nf = freqs.size
        F = torch.as_tensor(F, dtype=torch.complex128, device=self.device).contiguous()
        if F.shape != (self.n, nf):
            raise ValueError(f"F must be [n_nodes, nfreq] = {(self.n, nf)}")
        P = torch.zeros_like(F) if P0 is None else P0.clone().contiguous()
        infos = (hz_solve_info * nf)()
        code = lib().hz_solve_sweep(self.ctx, nf, _np_ptr(freqs, C.c_double), _dev(F, F.dtype),
                                    _dev(P, P.dtype), C.byref(make_opts(**opts)), infos)
        check(code)
        self.freq = None
        return P, [infos[j].as_dict() for j in range(nf)]

    def apply_sweep(self, freqs, X, precision="fp64"):
        """(Y, variant code): Y[:, c] = A(k_c) X[:, c] with the sweep's
        multi-vector product (hz_apply_sweep); X is [n_nodes, nfreq]."""
        import torch
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        nf = freqs.size
        X = torch.as_tensor(X, dtype=torch.complex128, device=self.device).contiguous()
        if X.shape != (self.n, nf):
            raise ValueError(f"X must be [n_nodes, nfreq] = {(self.n, nf)}")
        Y = torch.empty_like(X)
        v = C.c_int32()
        check(lib().hz_apply_sweep(self.ctx, nf, _np_ptr(freqs, C.c_double), PRECISIONS[precision],
                                   _dev(X, X.dtype), _dev(Y, Y.dtype), C.byref(v)), False)
        self.freq = None
        return Y, v.value

    def solve_adjoint(self, p, g, dJ_deta=None, **opts):
        """Returns (lambda, dJ_dbeta (6,2) numpy, info); dJ_deta (float64 device
        tensor of n_elems) is accumulated in place when given."""
        p = self._vec(p)
        g = self._vec(g)
        lam = self._vec()
        db = np.zeros(12, dtype=np.float64)
        info = hz_solve_info()
        de = None if dJ_deta is None else _dev(dJ_deta, dJ_deta.dtype)
        code = lib().hz_solve_adjoint(self.ctx, C.byref(make_opts(**opts)), _dev(p, p.dtype),
                                      _dev(g, g.dtype), _dev(lam, lam.dtype), _np_ptr(db, C.c_double),
                                      de, C.byref(info))
        check(code)
        return lam, db.reshape(6, 2), info.as_dict()
