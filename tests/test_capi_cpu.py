"""C-ABI contract checks that need no GPU: the library loads, exports every
function the header declares, and rejects bad input before touching HIP."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.cpu

hz = pytest.importorskip("paper_2112_00087_amd.hz")


@pytest.fixture(scope="module")
def L():
    return hz.lib()


def test_exports_every_header_symbol(L):
    import subprocess
    names = hz.header_symbols()
    assert {"hz_assemble", "hz_set_frequency", "hz_solve", "hz_solve_sweep", "hz_solve_adjoint"} <= set(names)
    for name in names:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", hz.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(names) <= exported


def _mesh_struct(mesh):
    keep = dict(xyz=np.ascontiguousarray(mesh["xyz"]), hex=np.ascontiguousarray(mesh["hex"], np.int32),
                bf=np.ascontiguousarray(mesh["bface"], np.int32),
                tag=np.ascontiguousarray(mesh["bface_tag"], np.int32),
                src=np.ascontiguousarray(mesh["bface_src"], np.uint8))
    m = hz.hz_mesh()
    m.n_nodes, m.n_elems, m.n_bfaces = keep["xyz"].shape[0], keep["hex"].shape[0], keep["bf"].shape[0]
    m.xyz = keep["xyz"].ctypes.data_as(C.POINTER(C.c_double))
    m.hex = keep["hex"].ctypes.data_as(C.POINTER(C.c_int32))
    m.bface = keep["bf"].ctypes.data_as(C.POINTER(C.c_int32))
    m.bface_tag = keep["tag"].ctypes.data_as(C.POINTER(C.c_int32))
    m.bface_src = keep["src"].ctypes.data_as(C.POINTER(C.c_uint8))
    m.c, m.rho = 340.0, 1.2
    return m, keep


def test_assemble_rejects_bad_input_without_gpu(L):
    out = C.c_void_p(1)
    beta = hz._beta_array(np.zeros(6))
    assert L.hz_assemble(None, beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    assert out.value is None
    assert "NULL" in hz.last_error()
    mesh = W.box_mesh(2, 2, 2)
    m, keep = _mesh_struct(mesh)
    keep["hex"][0, 3] = 10_000          # node id out of range
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    assert "out of range" in hz.last_error()
    m, keep = _mesh_struct(mesh)
    keep["tag"][0] = 7                  # wall id out of range
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    m, keep = _mesh_struct(mesh)
    keep["xyz"][3, 1] = np.nan
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    m, keep = _mesh_struct(mesh)
    m.c = -1.0
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    eta = np.full(mesh["n_elems"], np.inf)
    m, keep = _mesh_struct(mesh)
    assert L.hz_assemble(C.byref(m), beta, eta.ctypes.data_as(C.POINTER(C.c_double)), None,
                         C.byref(out)) == hz.HZ_ERR_INVALID
    # a face that is not an element face
    m, keep = _mesh_struct(mesh)
    keep["bf"][0] = [0, 2, 18, 26]
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID


def test_null_context_and_options(L):
    o = hz.make_opts()
    info = hz.hz_solve_info()
    assert L.hz_solve(None, C.byref(o), None, None, C.byref(info)) == hz.HZ_ERR_INVALID
    assert L.hz_set_frequency(None, 100.0) == hz.HZ_ERR_INVALID
    assert L.hz_sizes(None, None, None, None, None) == hz.HZ_ERR_INVALID
    L.hz_destroy(None)   # ignored


def test_opts_struct_layout_matches_header():
    # 6 int32, 2 double, hz_c128, 2 int32, hz_c128
    assert C.sizeof(hz.hz_solve_opts) == 6 * 4 + 2 * 8 + 16 + 2 * 4 + 16
    assert hz.hz_solve_opts.dd_alpha2.offset == 64
    assert C.sizeof(hz.hz_solve_info) == 4 * 4 + 3 * 8
    assert hz.hz_mesh.xyz.offset == 16
    # ..., elems[3], parts[3], order, sigma after c and rho
    assert hz.hz_mesh.order.offset == hz.hz_mesh.parts.offset + 12
    assert hz.hz_mesh.sigma.offset == hz.hz_mesh.order.offset + 4
    assert hz.hz_mesh.elem_type.offset == hz.hz_mesh.sigma.offset + 4


def _factor(lam, a0, a1):
    return np.max(np.abs((lam - a0) * (lam - a1) / ((lam + a0) * (lam + a1))))


def test_dd_alpha_optimiser_host_only():
    """The coefficient optimiser runs on the host (no GPU).  Checked against
    the convergence factor written out from its definition: the two-sided
    pair does at least as well as the one-sided coefficient used on both
    sides (whose double-step factor is the one-sided factor squared), and
    both beat the plain absorbing choice i k."""
    import paper_2112_00087_amd as P
    k, H, h = 2.772, 0.4, 0.01
    a1, b1 = P.dd_alpha(k, H, h, sides=1)
    a2, b2 = P.dd_alpha(k, H, h, sides=2)
    assert a1 == b1 and a1.real > 0 and a1.imag > 0
    assert a2.real > 0 and a2.imag > 0 and b2.real > 0 and b2.imag > 0
    xi = np.geomspace(np.pi / H, np.pi / h, 2000)
    xi = xi[np.abs(xi - k) > 0.5 * np.pi / H]
    lam = np.where(xi > k, np.sqrt(np.abs(xi ** 2 - k ** 2)) + 0j, 1j * np.sqrt(np.abs(k ** 2 - xi ** 2)))
    one, two, plain = _factor(lam, a1, a1), _factor(lam, a2, b2), _factor(lam, 1j * k, 1j * k)
    assert two <= one * (1 + 1e-12) and one < plain
    with pytest.raises(P.HzError):
        P.dd_alpha(k, 0.01, 0.4)
    with pytest.raises(P.HzError):
        P.dd_alpha(k, H, h, sides=3)


def _graph(mesh):
    import scipy.sparse as sp
    conn = mesh["tet"] if "tet" in mesh else mesh["hex"]
    ne, n, npe = conn.shape[0], mesh["xyz"].shape[0], conn.shape[1]
    E = sp.csr_matrix((np.ones(ne * npe), (np.repeat(np.arange(ne), npe), conn.ravel())), shape=(ne, n))
    G = (E.T @ E).tocsr()
    G.sort_indices()
    return G


def _bandwidth(G, perm):
    ip = np.empty_like(perm)
    ip[perm] = np.arange(perm.size)
    c = G.tocoo()
    return int(np.abs(ip[c.row] - ip[c.col]).max())


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_node_order_host_only(kind):
    """The internal numbering (host computation, no GPU): a permutation; the
    reverse Cuthill-McKee band is as narrow as scipy's implementation of the
    same method gives (an independent library routine) and far below the
    random input numbering's; the length sort leaves every window of sigma
    rows ordered by row length, longest first, holding the same nodes."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    import paper_2112_00087_amd as P
    mesh = W.kuhn_hex_mesh(6, 4, 4) if kind == "hex" else W.kuhn_tet_mesh(12, 8, 8)
    n = mesh["n_nodes"]
    G = _graph(mesh)
    rl = np.diff(G.indptr)
    ident = P.node_order(mesh, "given", 0)
    assert np.array_equal(ident, np.arange(n))
    rcm = P.node_order(mesh, "rcm", 0)
    assert np.array_equal(np.sort(rcm), np.arange(n))
    ref = np.asarray(reverse_cuthill_mckee(G, symmetric_mode=True))
    b_rcm, b_ref, b_in = _bandwidth(G, rcm), _bandwidth(G, ref), _bandwidth(G, ident)
    assert b_rcm <= 1.15 * b_ref and b_rcm < b_in / 5, (b_rcm, b_ref, b_in)
    for sigma in (64, 256):
        srt = P.node_order(mesh, "rcm", sigma)
        for w in range(0, n, sigma):
            a, b = rcm[w:w + sigma], srt[w:w + sigma]
            assert np.array_equal(np.sort(a), np.sort(b))
            assert np.all(np.diff(rl[b]) <= 0)
    # deterministic
    assert np.array_equal(P.node_order(mesh, "rcm", 256), P.node_order(mesh, "rcm", 256))
    # a structured box in lexicographic order stays a narrow band too
    box = W.box_mesh(6, 5, 4)
    Gb = _graph(box)
    assert _bandwidth(Gb, P.node_order(box, "rcm", 0)) <= 2 * _bandwidth(Gb, np.arange(box["n_nodes"]))
    with pytest.raises(P.HzError):
        P.node_order(mesh, "rcm", 100)          # not a multiple of 64
    with pytest.raises(P.HzError):
        P.node_order(mesh, 7, 0)


def test_assemble_rejects_reordered_schwarz_without_gpu(L):
    out = C.c_void_p(1)
    beta = hz._beta_array(np.zeros(6))
    m, keep = _mesh_struct(W.box_mesh(2, 2, 2))
    m.elems[:] = (2, 2, 2)
    m.parts[:] = (2, 1, 1)
    m.order = 1
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    assert "numbering" in hz.last_error()
    m.order, m.sigma = 0, 96
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID


def test_assemble_rejects_bad_element_type_without_gpu(L):
    out = C.c_void_p(1)
    beta = hz._beta_array(np.zeros(6))
    m, keep = _mesh_struct(W.box_mesh(2, 2, 2))
    m.elem_type = 2
    assert L.hz_assemble(C.byref(m), beta, None, None, C.byref(out)) == hz.HZ_ERR_INVALID
    assert "element type" in hz.last_error()
    # tetrahedra with a node id out of range (4 ids per element are read)
    t = W.kuhn_tet_mesh(2, 2, 1)
    conn = np.ascontiguousarray(t["tet"], np.int32)
    conn[-1, 3] = t["n_nodes"]
    m2 = hz.hz_mesh()
    m2.n_nodes, m2.n_elems = t["n_nodes"], conn.shape[0]
    m2.hex = conn.ctypes.data_as(C.POINTER(C.c_int32))
    m2.elem_type = hz.HZ_TET4
    perm = np.empty(t["n_nodes"], np.int32)
    assert L.hz_node_order(C.byref(m2), perm.ctypes.data_as(C.POINTER(C.c_int32))) == hz.HZ_ERR_INVALID
    assert "out of range" in hz.last_error()
