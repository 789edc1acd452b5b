"""Host-side checks of the C ABI (no GPU needed).

The library loads without a device, exports every function declared in
include/tdfe.h, validates arguments on the host and reports call-order
errors before touching the device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1810_13130_amd import tdfe
    if not os.path.exists(tdfe.LIB_PATH):
        pytest.skip("libtdfe.so not built")
    return tdfe.load()


def _declared():
    txt = open(os.path.join(ROOT, "include", "tdfe.h")).read()
    return sorted(set(re.findall(r"\b(tdfe_[a-zA-Z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "tdfe_magnus_step" in names and "tdfe_apply_H" in names
    for n in names:
        assert hasattr(lib, n), n


def _desc(tdfe, p=2, nc=(2, 2, 2), nq=None, k_max=16, n_orb=2, vertices=None, precision=0):
    d = tdfe.MeshDesc()
    d.p = p
    d.nq = p + 1 if nq is None else nq
    d.ncell[0], d.ncell[1], d.ncell[2] = nc
    v = W.box_vertices(-1.0, 1.0, nc).reshape(-1) if vertices is None else vertices
    v = np.ascontiguousarray(v, dtype=np.float64)
    d.vertices = v.ctypes.data_as(tdfe._DP)
    d.n_orb_max = n_orb
    d.k_max = k_max
    d.precision = precision
    return d, v


def _setup(lib, d):
    h = ctypes.c_void_p()
    s = lib.tdfe_fe_mesh_setup(ctypes.byref(d), None, ctypes.byref(h))
    return s, h


@pytest.mark.parametrize("kw", [dict(p=0), dict(p=9), dict(nq=4), dict(nc=(0, 2, 2)), dict(k_max=0),
                                dict(k_max=2000), dict(n_orb=0), dict(precision=7), dict(p=1, nc=(1, 2, 2))])
def test_setup_rejects_bad_descriptions(lib, kw):
    from paper_1810_13130_amd import tdfe
    d, keep = _desc(tdfe, **kw)
    s, h = _setup(lib, d)
    assert s == tdfe.EINVAL and not h.value


def test_matrix_core_precisions_need_box_cells_and_their_order_limit(lib):
    from paper_1810_13130_amd import tdfe
    curved = W.box_vertices(-1.0, 1.0, (2, 2, 2)).copy()
    curved[1, 1, 1, 0] += 0.1  # one interior vertex moved: trilinear cells
    for prec, p_max in ((tdfe.FP32_MFMA, 7), (tdfe.BF16_MFMA, 7), (tdfe.FP64_MFMA, 6)):
        d, keep = _desc(tdfe, p=p_max, precision=prec)
        s, h = _setup(lib, d)
        assert s == tdfe.OK
        lib.tdfe_destroy(h)
        d, keep = _desc(tdfe, p=p_max + 1, precision=prec)
        assert _setup(lib, d)[0] == tdfe.EINVAL
        d, keep = _desc(tdfe, p=2, precision=prec, vertices=curved.reshape(-1))
        assert _setup(lib, d)[0] == tdfe.EINVAL


def test_setup_rejects_nonfinite_vertex(lib):
    from paper_1810_13130_amd import tdfe
    v = W.box_vertices(-1.0, 1.0, (2, 2, 2)).reshape(-1).copy()
    v[5] = np.nan
    d, keep = _desc(tdfe, vertices=v)
    assert _setup(lib, d)[0] == tdfe.EINVAL


def test_query_sizes_and_call_order(lib):
    from paper_1810_13130_amd import tdfe
    d, keep = _desc(tdfe, p=3, nc=(2, 3, 4))
    s, h = _setup(lib, d)
    assert s == tdfe.OK
    nd, nc, nq, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    assert lib.tdfe_query(h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nq), ctypes.byref(ws)) == 0
    assert nd.value == 5 * 8 * 11 and nc.value == 24 and nq.value == 24 * 64 and ws.value > 0
    buf = ctypes.c_void_p(4096)  # never dereferenced: the calls must fail on the host first
    assert lib.tdfe_apply_H(h, buf, ctypes.c_void_p(8192), 1) == tdfe.ESTATE
    assert lib.tdfe_apply_H(h, buf, buf, 1) == tdfe.EINVAL
    assert lib.tdfe_apply_H(h, buf, ctypes.c_void_p(8192), 3) == tdfe.EINVAL
    assert lib.tdfe_dof_coords(h, buf) == tdfe.ESTATE
    assert lib.tdfe_lanczos_expm(h, buf, 1, 0.1, 0.0, None, None) == tdfe.EINVAL
    assert lib.tdfe_lanczos_expm(h, buf, 1, 0.1, 1e-8, None, None) == tdfe.ESTATE
    assert lib.tdfe_magnus_step(h, buf, 1, -0.1, 0.0, 1e-8, None) == tdfe.EINVAL
    assert lib.tdfe_magnus_step(h, buf, 1, 0.1, 0.0, 1e-8, None) == tdfe.ESTATE
    assert lib.tdfe_propagate(h, buf, 1, 0, 0.1, None, 1e-8, None, None) == tdfe.EINVAL
    bad_E = (ctypes.c_double * 2)(0.0, float("nan"))
    assert lib.tdfe_propagate(h, buf, 1, 2, 0.1, bad_E, 1e-8, None, None) == tdfe.EINVAL
    assert lib.tdfe_propagate(h, buf, 1, 2, 0.1, None, 1e-8, None, None) == tdfe.ESTATE
    assert b"before" in lib.tdfe_last_error(h)
    nb = ctypes.c_size_t()
    assert lib.tdfe_gradient_query(h, 1, 4, 2, 8, ctypes.byref(nb)) == tdfe.ESTATE
    assert lib.tdfe_gradient_query(h, 1, 4, 2, 8, None) == tdfe.EINVAL
    E = (ctypes.c_double * 4)()
    L, g = ctypes.c_double(), (ctypes.c_double * 4)()
    assert lib.tdfe_dipole_gradient(h, None, 1, 4, E, 0.1, 1e-8, 2, 8, buf, 1 << 20, ctypes.byref(L), g) == tdfe.EINVAL
    assert lib.tdfe_dipole_gradient(h, buf, 1, 4, E, 0.1, 1e-8, 2, 8, buf, 1 << 20, ctypes.byref(L), g) == tdfe.ESTATE
    # Kleinman-Bylander store: Cbar (n_proj x n_dof FP64) plus scratch; set only after bind
    pb = ctypes.c_size_t()
    assert lib.tdfe_projector_query(h, 4, ctypes.byref(pb)) == 0
    assert pb.value >= 4 * nd.value * 8 + nq.value * 8
    assert lib.tdfe_projector_query(h, 0, ctypes.byref(pb)) == 0 and pb.value == 0
    assert lib.tdfe_projector_query(h, -1, ctypes.byref(pb)) == tdfe.EINVAL
    assert lib.tdfe_projector_query(h, 1025, ctypes.byref(pb)) == tdfe.EINVAL
    assert lib.tdfe_projector_query(h, 4, None) == tdfe.EINVAL
    assert lib.tdfe_set_projectors(h, 4, buf, buf, buf, 1 << 30) == tdfe.ESTATE
    md = tdfe.MidpointDesc()
    for mode, order, tol_, it in ((5, 1, 1e-10, 10), (1, 3, 1e-10, 10), (1, 1, 0.0, 10), (1, 1, 1e-10, 0),
                                  (1, 1, float("nan"), 10)):
        md.mode, md.order, md.sc_tol, md.sc_maxit = mode, order, tol_, it
        assert lib.tdfe_set_midpoint(h, ctypes.byref(md)) == tdfe.EINVAL
    md.mode, md.order, md.sc_tol, md.sc_maxit = 1, 2, 1e-10, 10
    assert lib.tdfe_set_midpoint(h, ctypes.byref(md)) == 0
    md.mode, md.order = 0, 1
    assert lib.tdfe_set_midpoint(h, ctypes.byref(md)) == 0
    ng, st, bd, ld = ctypes.c_int(7), ctypes.c_int64(7), ctypes.c_int64(7), ctypes.c_int64(7)
    assert lib.tdfe_projector_info(h, ctypes.byref(ng), ctypes.byref(st), ctypes.byref(bd), ctypes.byref(ld)) == 0
    assert (ng.value, st.value, bd.value, ld.value) == (0, 0, 0, 0)
    assert lib.tdfe_projector_info(h, ctypes.byref(ng), ctypes.byref(st), ctypes.byref(bd), None) == tdfe.EINVAL
    assert lib.tdfe_bind_workspace(h, None, 0) == tdfe.EINVAL
    assert lib.tdfe_bind_workspace(h, ctypes.c_void_p(4096 + 8), ws.value) == tdfe.EINVAL
    assert lib.tdfe_bind_workspace(h, ctypes.c_void_p(4096), ws.value - 1) == tdfe.ENOMEM
    lib.tdfe_destroy(h)


def test_soft_chunk_query_before_any_exponential(lib, monkeypatch):
    """With the basis memory capped at two orbitals, eight orbitals run in
    chunks of two at k_max until an exponential has shown its Krylov
    dimension; the workspace holds the widest soft-capped chunk's operator
    output (seven orbitals: (128 + 1) 2 / 7 - 1 = 35 >= 32 vectors)."""
    from paper_1810_13130_amd import tdfe
    sizes = {}
    for env in ("TDFE_BASIS_CHUNK_ORB", "TDFE_MAX_CHUNK_ORB"):
        monkeypatch.delenv("TDFE_BASIS_CHUNK_ORB", raising=False)
        monkeypatch.delenv("TDFE_MAX_CHUNK_ORB", raising=False)
        monkeypatch.setenv(env, "2")
        d, keep = _desc(tdfe, p=2, nc=(2, 2, 2), k_max=128, n_orb=8)
        s, h = _setup(lib, d)
        assert s == tdfe.OK
        ch, cap = ctypes.c_int(), ctypes.c_int()
        assert lib.tdfe_krylov_chunk(h, 8, ctypes.byref(ch)) == 0 and ch.value == 2
        assert lib.tdfe_krylov_soft_chunk(h, 8, ctypes.byref(ch), ctypes.byref(cap)) == 0
        assert (ch.value, cap.value) == (2, 128)
        assert lib.tdfe_krylov_soft_chunk(h, 0, ctypes.byref(ch), ctypes.byref(cap)) == tdfe.EINVAL
        assert lib.tdfe_krylov_soft_chunk(h, 9, ctypes.byref(ch), ctypes.byref(cap)) == tdfe.EINVAL
        assert lib.tdfe_krylov_soft_chunk(h, 8, None, ctypes.byref(cap)) == tdfe.EINVAL
        assert lib.tdfe_krylov_soft_chunk(h, 8, ctypes.byref(ch), None) == tdfe.EINVAL
        nd, nc, nq, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        assert lib.tdfe_query(h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nq), ctypes.byref(ws)) == 0
        sizes[env] = (ws.value, nd.value)
        lib.tdfe_destroy(h)
    assert lib.tdfe_krylov_soft_chunk(None, 8, ctypes.byref(ch), ctypes.byref(cap)) == tdfe.EINVAL
    # the operator output for 7 orbitals instead of 2: at least 10 more columns per DoF
    (wb, nd), (wm, _) = sizes["TDFE_BASIS_CHUNK_ORB"], sizes["TDFE_MAX_CHUNK_ORB"]
    assert wb - wm >= 10 * nd * 8


def test_null_arguments(lib):
    from paper_1810_13130_amd import tdfe
    assert lib.tdfe_fe_mesh_setup(None, None, None) == tdfe.EINVAL
    assert lib.tdfe_query(None, None, None, None, None) == tdfe.EINVAL
    assert lib.tdfe_last_error(None) == b"null context"
