"""Thin Python binding of the tdfe C ABI (include/tdfe.h).

Argument marshalling only: every step of the method runs in the HIP library
``libtdfe.so`` built from ``csrc/``.  PyTorch supplies device memory and the
HIP stream.  There is no fallback: if the library is missing, loading fails.

Function names match the C ABI without the ``tdfe_`` prefix; ``Context``
bundles a context with its torch-owned workspace.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdfe.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESTATE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED_FP32 = 0, 1
# matrix-core variants of the cell operator (box meshes): FP32 storage for the
# first two (as MIXED_FP32), FP64 for the third
FP32_MFMA, BF16_MFMA, FP64_MFMA = 2, 3, 4
XC_NONE, XC_X, XC_XC = 0, 1, 2
PCG_FDM, PCG_JACOBI = 0, 1
_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "ESTATE", -6: "ENONFINITE"}


class TdfeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tdfe status {status} ({_NAMES.get(status, '?')}): {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("nq", ctypes.c_int), ("ncell", ctypes.c_int * 3),
                ("vertices", ctypes.POINTER(ctypes.c_double)), ("n_orb_max", ctypes.c_int),
                ("k_max", ctypes.c_int), ("precision", ctypes.c_int)]


class ScfDesc(ctypes.Structure):
    _fields_ = [("hartree", ctypes.c_int), ("xc", ctypes.c_int), ("n_nuclei", ctypes.c_int),
                ("Z", ctypes.POINTER(ctypes.c_double)), ("R", ctypes.POINTER(ctypes.c_double)),
                ("occupation", ctypes.POINTER(ctypes.c_double)), ("n_orb", ctypes.c_int),
                ("pcg_tol", ctypes.c_double), ("pcg_maxit", ctypes.c_int), ("pcg_precond", ctypes.c_int)]


class StepReport(ctypes.Structure):
    _fields_ = [("k_pred_max", ctypes.c_int), ("k_corr_max", ctypes.c_int), ("k_pred_sum", ctypes.c_int),
                ("k_corr_sum", ctypes.c_int), ("err_max", ctypes.c_double), ("poisson_iters", ctypes.c_int),
                ("mu", ctypes.c_double * 3), ("charge", ctypes.c_double), ("sc_iters", ctypes.c_int),
                ("sc_change", ctypes.c_double)]

    def as_dict(self):
        return {"k_pred_max": self.k_pred_max, "k_corr_max": self.k_corr_max, "k_pred_sum": self.k_pred_sum,
                "k_corr_sum": self.k_corr_sum, "err_max": self.err_max, "poisson_iters": self.poisson_iters,
                "mu": np.array(self.mu[:]), "charge": self.charge, "sc_iters": self.sc_iters,
                "sc_change": self.sc_change}


class AdaptDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("n_atoms", ctypes.c_int),
                ("R", ctypes.POINTER(ctypes.c_double)), ("Z", ctypes.POINTER(ctypes.c_double)),
                ("s_orb", ctypes.POINTER(ctypes.c_double)), ("a_pot", ctypes.POINTER(ctypes.c_double)),
                ("n_elem", ctypes.c_double), ("samples", ctypes.c_int)]


class OctreeDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("n0", ctypes.c_int),
                ("max_level", ctypes.c_int), ("n_leaf", ctypes.c_int), ("leaves", ctypes.POINTER(ctypes.c_int)),
                ("n_orb_max", ctypes.c_int), ("k_max", ctypes.c_int), ("precision", ctypes.c_int)]


class MidpointDesc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("order", ctypes.c_int), ("sc_tol", ctypes.c_double),
                ("sc_maxit", ctypes.c_int)]


MIDPOINT_PC = 0
MIDPOINT_SC = 1


_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
SIGNATURES = {
    "tdfe_fe_mesh_setup": [ctypes.POINTER(MeshDesc), _P, ctypes.POINTER(_P)],
    "tdfe_query": [_P, _I64P, _I64P, _I64P, ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_bind_workspace": [_P, _P, ctypes.c_size_t],
    "tdfe_dof_coords": [_P, _P],
    "tdfe_quad_coords": [_P, _P],
    "tdfe_mass_diag": [_P, _P],
    "tdfe_set_potential": [_P, _P],
    "tdfe_set_scf": [_P, ctypes.POINTER(ScfDesc)],
    "tdfe_projector_query": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_set_projectors": [_P, ctypes.c_int, _P, _P, _P, ctypes.c_size_t],
    "tdfe_projector_info": [_P, _IP, _I64P, _I64P, _I64P],
    "tdfe_set_field_direction": [_P, _DP],
    "tdfe_set_midpoint": [_P, ctypes.POINTER(MidpointDesc)],
    "tdfe_adaptive_axes_query": [ctypes.POINTER(AdaptDesc), ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_adaptive_axes": [ctypes.POINTER(AdaptDesc), _P, ctypes.c_size_t, _P, ctypes.c_int, _DP, _IP, _DP],
    "tdfe_adaptive_axes_static": [ctypes.POINTER(AdaptDesc), _P, ctypes.c_int, _DP, _IP, _DP],
    "tdfe_octree_leaves_query": [ctypes.POINTER(AdaptDesc), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_octree_leaves": [ctypes.POINTER(AdaptDesc), ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _P,
                           ctypes.c_int, _IP, _IP, _DP],
    "tdfe_fe_octree_setup": [ctypes.POINTER(OctreeDesc), _P, ctypes.POINTER(_P)],
    "tdfe_octree_info": [_P, _I64P, _I64P, _I64P],
    "tdfe_tridiag_expm_query": [ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_tridiag_expm": [_P, _P, ctypes.c_int, ctypes.c_double, _P, _P, ctypes.c_size_t, _P, _IP],
    "tdfe_kick": [_P, _P, ctypes.c_int, ctypes.c_double],
    "tdfe_field_samples": [ctypes.c_int, _DP, ctypes.c_int, _DP, _DP],
    "tdfe_absorption_spectrum": [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P,
                                 ctypes.c_int, _P, _P],
    "tdfe_power_spectrum": [_P, ctypes.c_int, ctypes.c_double, _P, ctypes.c_int, _P, _P],
    "tdfe_apply_H": [_P, _P, _P, ctypes.c_int],
    "tdfe_apply_H_add": [_P, _P, _P, ctypes.c_int],
    "tdfe_apply_H_add_f32": [_P, _P, _P, ctypes.c_int],
    "tdfe_lanczos_expm": [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _IP, _DP],
    "tdfe_density": [_P, _P, ctypes.c_int, _P],
    "tdfe_krylov_chunk": [_P, ctypes.c_int, _IP],
    "tdfe_krylov_soft_chunk": [_P, ctypes.c_int, _IP, _IP],
    "tdfe_scf_fields": [_P, _P, ctypes.c_int, _P, _P],
    "tdfe_dipole": [_P, _P, ctypes.c_int, _DP, _DP],
    "tdfe_magnus_step": [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                         ctypes.POINTER(StepReport)],
    "tdfe_propagate": [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _DP, ctypes.c_double, _P,
                       ctypes.POINTER(StepReport)],
    "tdfe_gradient_query": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_size_t)],
    "tdfe_dipole_gradient": [_P, _P, ctypes.c_int, ctypes.c_int, _DP, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _DP, _DP],
    "tdfe_last_error": [_P],
    "tdfe_destroy": [_P],
}

_lib = None


def load(path=LIB_PATH):
    """Load libtdfe.so and declare every exported function; raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libtdfe.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.tdfe_last_error.restype = ctypes.c_char_p
    lib.tdfe_destroy.restype = None
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One tdfe context plus its torch-owned workspace on the current device."""

    def __init__(self, p, ncell, vertices, n_orb_max, k_max=128, precision=FP64, nq=None, stream=None):
        import torch
        self.lib = load()
        v = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64).reshape(-1))
        self._vert = v
        d = MeshDesc()
        d.p = p
        d.nq = p + 1 if nq is None else nq
        d.ncell[0], d.ncell[1], d.ncell[2] = ncell
        d.vertices = v.ctypes.data_as(_DP)
        d.n_orb_max = n_orb_max
        d.k_max = k_max
        d.precision = precision
        self._stream = stream if stream is not None else _stream_handle()
        h = ctypes.c_void_p()
        s = self.lib.tdfe_fe_mesh_setup(ctypes.byref(d), self._stream, ctypes.byref(h))
        if s != OK:
            raise TdfeError(s, "fe_mesh_setup rejected the mesh description")
        self.h = h
        self.p, self.nq = p, d.nq
        self.n_nodes = int(np.prod([c * p + 1 for c in ncell]))
        self._bind(n_orb_max)

    def _bind(self, n_orb_max):
        import torch
        self.n_dof, self.n_cell, self.n_quad, self.ws_bytes = self.query()
        self.n_orb_max = n_orb_max
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._check(self.lib.tdfe_bind_workspace(self.h, ctypes.c_void_p(base + off), self.ws_bytes))

    @classmethod
    def octree(cls, p, lo, hi, n0, max_level, leaves, n_orb_max, k_max=128, stream=None):
        """A context on the leaves ({q, i, j, k} rows) of an octree over
        [lo, hi]^3 with hanging-node constraints (tdfe_fe_octree_setup)."""
        self = cls.__new__(cls)
        self.lib = load()
        lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        self._leaves = lv
        d = OctreeDesc()
        d.p, d.lo, d.hi, d.n0, d.max_level = p, lo, hi, n0, max_level
        d.n_leaf = len(lv)
        d.leaves = lv.ctypes.data_as(_IP)
        d.n_orb_max, d.k_max, d.precision = n_orb_max, k_max, FP64
        self._stream = stream if stream is not None else _stream_handle()
        h = ctypes.c_void_p()
        s = self.lib.tdfe_fe_octree_setup(ctypes.byref(d), self._stream, ctypes.byref(h))
        if s != OK:
            raise TdfeError(s, "fe_octree_setup rejected the octree")
        self.h = h
        self.p, self.nq = p, p + 1
        nn, nh, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tdfe_octree_info(self.h, ctypes.byref(nn), ctypes.byref(nh), ctypes.byref(nz)))
        self.n_nodes, self.n_hanging, self.constraint_nnz = nn.value, nh.value, nz.value
        self._bind(n_orb_max)
        return self

    # -- plumbing ---------------------------------------------------------------
    def _check(self, s):
        if s != OK:
            raise TdfeError(s, self.lib.tdfe_last_error(self.h).decode())
        return s

    def close(self):
        """destroy the context and drop its workspace (the memory returns to
        torch's caching allocator at once, not when this object is collected)"""
        if getattr(self, "h", None):
            self.lib.tdfe_destroy(self.h)
            self.h = None
        self.workspace = None
        self._nl_store = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls (same names as the C functions) -----------------------------------
    def query(self):
        nd, nc, nq = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ws = ctypes.c_size_t()
        self._check(self.lib.tdfe_query(self.h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nq),
                                        ctypes.byref(ws)))
        return nd.value, nc.value, nq.value, ws.value

    def dof_coords(self):
        import torch
        out = torch.empty((self.n_dof, 3), dtype=torch.float64, device="cuda")
        self._check(self.lib.tdfe_dof_coords(self.h, _ptr(out)))
        return out

    def quad_coords(self):
        import torch
        out = torch.empty((self.n_cell, self.n_quad // self.n_cell, 3), dtype=torch.float64, device="cuda")
        self._check(self.lib.tdfe_quad_coords(self.h, _ptr(out)))
        return out

    def mass_diag(self):
        import torch
        out = torch.empty(self.n_dof, dtype=torch.float64, device="cuda")
        self._check(self.lib.tdfe_mass_diag(self.h, _ptr(out)))
        return out

    def set_potential(self, v):
        assert v.dtype.is_floating_point and v.numel() == self.n_quad and v.is_contiguous()
        self._check(self.lib.tdfe_set_potential(self.h, _ptr(v)))

    def set_scf(self, hartree=False, xc=XC_NONE, Z=(), R=(), occupation=None, n_orb=0, pcg_tol=1e-13,
                pcg_maxit=5000, pcg_precond=None):
        """pcg_precond (curved meshes): PCG_FDM (default) or PCG_JACOBI."""
        s = ScfDesc()
        s.hartree = int(bool(hartree))
        s.xc = xc
        Zc = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).reshape(-1))
        Rc = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(-1))
        self._scf_keep = [Zc, Rc]
        s.n_nuclei = len(Zc)
        s.Z = Zc.ctypes.data_as(_DP)
        s.R = Rc.ctypes.data_as(_DP)
        if occupation is not None:
            oc = np.ascontiguousarray(np.asarray(occupation, dtype=np.float64))
            self._scf_keep.append(oc)
            s.occupation = oc.ctypes.data_as(_DP)
            s.n_orb = len(oc)
        else:
            s.n_orb = n_orb
        s.pcg_tol = pcg_tol
        s.pcg_maxit = pcg_maxit
        s.pcg_precond = PCG_FDM if pcg_precond is None else pcg_precond
        self._check(self.lib.tdfe_set_scf(self.h, ctypes.byref(s)))

    def projector_query(self, n_proj):
        b = ctypes.c_size_t()
        self._check(self.lib.tdfe_projector_query(self.h, n_proj, ctypes.byref(b)))
        return b.value

    def set_projectors(self, u, dv):
        """Kleinman-Bylander term from u_p and dV_p at the Gauss points
        ([n_proj][n_cell][nq^3] FP64 device tensors); u = None removes it.
        The device store is a torch tensor held by this object."""
        import torch
        if u is None:
            self._check(self.lib.tdfe_set_projectors(self.h, 0, None, None, None, 0))
            self._nl_store = None
            return
        assert u.dtype == torch.float64 and dv.dtype == torch.float64 and u.is_cuda and dv.is_cuda
        assert u.is_contiguous() and dv.is_contiguous() and u.shape == dv.shape
        n_proj = u.shape[0]
        assert u.numel() == n_proj * self.n_quad
        nbytes = self.projector_query(n_proj)
        store = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = store.data_ptr()
        off = (-base) % 256
        self._check(self.lib.tdfe_set_projectors(self.h, n_proj, _ptr(u), _ptr(dv),
                                                 ctypes.c_void_p(base + off), nbytes))
        self._nl_store = store

    def projector_info(self):
        """(groups, stored entries of Cbar, DoFs in the boxes, DoFs on the crossed lines)."""
        g, st, bd, ld = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.tdfe_projector_info(self.h, ctypes.byref(g), ctypes.byref(st), ctypes.byref(bd),
                                                 ctypes.byref(ld)))
        return g.value, st.value, bd.value, ld.value

    def set_midpoint(self, mode=MIDPOINT_PC, order=1, sc_tol=1e-10, sc_maxit=50):
        m = MidpointDesc()
        m.mode, m.order, m.sc_tol, m.sc_maxit = mode, order, sc_tol, sc_maxit
        self._check(self.lib.tdfe_set_midpoint(self.h, ctypes.byref(m)))

    def set_field_direction(self, d):
        dd = (ctypes.c_double * 3)(*[float(v) for v in d])
        self._check(self.lib.tdfe_set_field_direction(self.h, dd))

    def kick(self, psibar, kappa):
        n_orb = self._orb(psibar)
        self._check(self.lib.tdfe_kick(self.h, _ptr(psibar), n_orb, float(kappa)))

    @staticmethod
    def _orb(psi):
        import torch
        assert psi.dtype == torch.complex128 and psi.is_contiguous() and psi.is_cuda
        return psi.shape[1]

    def apply_H(self, psibar, out=None):
        import torch
        n = self._orb(psibar)
        if out is None:
            out = torch.empty_like(psibar)
        self._check(self.lib.tdfe_apply_H(self.h, _ptr(psibar), _ptr(out), n))
        return out

    def apply_H_add(self, psibar, out):
        n = self._orb(psibar)
        self._check(self.lib.tdfe_apply_H_add(self.h, _ptr(psibar), _ptr(out), n))
        return out

    def apply_H_add_f32(self, psibar, out):
        import torch
        assert psibar.dtype == torch.complex64 and out.dtype == torch.complex64
        self._check(self.lib.tdfe_apply_H_add_f32(self.h, _ptr(psibar), _ptr(out), psibar.shape[1]))
        return out

    def lanczos_expm(self, psibar, tau, tol):
        n = self._orb(psibar)
        ks = (ctypes.c_int * n)()
        es = (ctypes.c_double * n)()
        self._check(self.lib.tdfe_lanczos_expm(self.h, _ptr(psibar), n, tau, tol, ks, es))
        return list(ks), list(es)

    def density(self, psibar, out=None):
        import torch
        n = self._orb(psibar)
        if out is None:
            out = torch.empty((self.n_cell, self.n_quad // self.n_cell), dtype=torch.float64, device="cuda")
        self._check(self.lib.tdfe_density(self.h, _ptr(psibar), n, _ptr(out)))
        return out

    def krylov_chunk(self, n_orb):
        """orbitals per Krylov chunk (one operator launch) for a call on n_orb orbitals"""
        k = ctypes.c_int()
        self._check(self.lib.tdfe_krylov_chunk(self.h, n_orb, ctypes.byref(k)))
        return k.value

    def krylov_soft_chunk(self, n_orb):
        """(chunk, Krylov dimension limit) of the next exponential on n_orb
        orbitals: wider chunks under a soft cap once an exponential has run"""
        k, cap = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tdfe_krylov_soft_chunk(self.h, n_orb, ctypes.byref(k), ctypes.byref(cap)))
        return k.value, cap.value

    def scf_fields(self, psibar, phi=True, w=True):
        """(phi over every grid node or None, W = V_H + V_xc at the Gauss points
        [n_cell][nq^3] or None) of the density of psibar; nothing is propagated."""
        import torch
        n = self._orb(psibar)
        ph = torch.empty(self.n_nodes, dtype=torch.float64, device="cuda") if phi else None
        wq = torch.empty((self.n_cell, self.n_quad // self.n_cell), dtype=torch.float64, device="cuda") if w else None
        self._check(self.lib.tdfe_scf_fields(self.h, _ptr(psibar), n, _ptr(ph) if ph is not None else None,
                                             _ptr(wq) if wq is not None else None))
        return ph, wq

    def dipole(self, psibar):
        n = self._orb(psibar)
        mu = (ctypes.c_double * 3)()
        ch = ctypes.c_double()
        self._check(self.lib.tdfe_dipole(self.h, _ptr(psibar), n, mu, ctypes.byref(ch)))
        return np.array(mu[:]), ch.value

    def magnus_step(self, psibar, dt, field_E=0.0, tol=1e-10, report=True):
        n = self._orb(psibar)
        rep = StepReport()
        self._check(self.lib.tdfe_magnus_step(self.h, _ptr(psibar), n, dt, field_E, tol,
                                              ctypes.byref(rep) if report else None))
        return rep.as_dict() if report else None

    def propagate(self, psibar, n_steps, dt, E=None, tol=1e-10, record=True):
        """n_steps Magnus steps in one call; returns (records [n_steps][4] =
        charge, mu_x, mu_y, mu_z per step as a device tensor or None, totals)."""
        import torch
        n = self._orb(psibar)
        Eh = None
        if E is not None:
            Eh = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1))
            assert Eh.size == n_steps
        mu = torch.empty((n_steps, 4), dtype=torch.float64, device="cuda") if record else None
        rep = StepReport()
        self._check(self.lib.tdfe_propagate(self.h, _ptr(psibar), n, n_steps, dt,
                                            Eh.ctypes.data_as(_DP) if Eh is not None else None, tol,
                                            _ptr(mu) if mu is not None else None, ctypes.byref(rep)))
        return mu, rep.as_dict()

    def gradient_query(self, n_orb, n_steps, checkpoint_every, k_store):
        b = ctypes.c_size_t()
        self._check(self.lib.tdfe_gradient_query(self.h, n_orb, n_steps, checkpoint_every, k_store, ctypes.byref(b)))
        return b.value

    def dipole_gradient(self, psibar0, E, dt, tol=1e-10, checkpoint_every=None, k_store=64):
        """(L, dL/dE) for L = mu_z after len(E) Magnus steps with fields E (numpy, float64)."""
        import torch
        n = self._orb(psibar0)
        E = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1))
        N = len(E)
        ck = N if checkpoint_every is None else int(checkpoint_every)
        nb = self.gradient_query(n, N, ck, k_store)
        work = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
        base = work.data_ptr()
        off = (-base) % 256
        L = ctypes.c_double()
        g = np.zeros(N, dtype=np.float64)
        self._check(self.lib.tdfe_dipole_gradient(self.h, _ptr(psibar0), n, N, E.ctypes.data_as(_DP), dt, tol, ck,
                                                  k_store, ctypes.c_void_p(base + off), nb, ctypes.byref(L),
                                                  g.ctypes.data_as(_DP)))
        del work
        return L.value, g


def _dipole_function():
    import torch

    class DipoleOfField(torch.autograd.Function):
        """L = mu_z(t_N) as a differentiable function of the field amplitudes.

        forward(E, ctx, psibar0, dt, tol, checkpoint_every, k_store): E is a
        float64 tensor of per-step amplitudes; the reverse sweep runs in the
        same library call as the forward one, so backward only scales the
        stored gradient.
        """

        @staticmethod
        def forward(fctx, E, ctx, psibar0, dt, tol=1e-10, checkpoint_every=None, k_store=64):
            L, g = ctx.dipole_gradient(psibar0, E.detach().cpu().numpy(), dt, tol, checkpoint_every, k_store)
            fctx.save_for_backward(torch.from_numpy(g).to(E.device))
            return torch.tensor(L, dtype=torch.float64, device=E.device)

        @staticmethod
        def backward(fctx, gL):
            (g,) = fctx.saved_tensors
            return gL * g, None, None, None, None, None, None

    return DipoleOfField


_DIPOLE_FN = None


def dipole_of_field(E, ctx, psibar0, dt, tol=1e-10, checkpoint_every=None, k_store=64):
    """Autograd entry: returns L (0-d tensor); L.backward() fills E.grad with dL/dE."""
    global _DIPOLE_FN
    if _DIPOLE_FN is None:
        _DIPOLE_FN = _dipole_function()
    return _DIPOLE_FN.apply(E, ctx, psibar0, dt, tol, checkpoint_every, k_store)


FIELD_GAUSSIAN = 1
FIELD_SIN2 = 2


def field_samples(shape, params, t):
    """E(t) for TDFE_FIELD_GAUSSIAN {kappa, t0, w} or TDFE_FIELD_SIN2 {kappa, omega, T}."""
    lib = load()
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    tt = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(-1))
    out = np.empty_like(tt)
    s = lib.tdfe_field_samples(int(shape), p.ctypes.data_as(_DP), tt.size, tt.ctypes.data_as(_DP),
                               out.ctypes.data_as(_DP))
    if s != OK:
        raise TdfeError(s, "field_samples: bad shape or parameters")
    return out


def absorption_spectrum(mu, dt, omega, alpha, kappa=None, field=None):
    """S(w) on the device: mu [3][n_t] (row a: a-component of the run excited
    along a), omega [n_w], field [3][n_t] or a kick strength kappa."""
    import torch
    lib = load()
    assert mu.dtype == torch.float64 and mu.is_cuda and mu.is_contiguous() and mu.shape[0] == 3
    assert omega.dtype == torch.float64 and omega.is_cuda and omega.is_contiguous()
    if field is not None:
        assert field.dtype == torch.float64 and field.is_cuda and field.is_contiguous() and field.shape == mu.shape
    out = torch.empty_like(omega)
    s = lib.tdfe_absorption_spectrum(_ptr(mu), _ptr(field) if field is not None else None, mu.shape[1], float(dt),
                                     float(kappa) if kappa is not None else 0.0, float(alpha), _ptr(omega),
                                     omega.numel(), _ptr(out), _stream_handle())
    if s != OK:
        raise TdfeError(s, "absorption_spectrum: bad arguments")
    return out


def power_spectrum(mu, dt, omega):
    """P(w) on the device from one dipole component mu [n_t]."""
    import torch
    lib = load()
    assert mu.dtype == torch.float64 and mu.is_cuda and mu.is_contiguous() and mu.dim() == 1
    assert omega.dtype == torch.float64 and omega.is_cuda and omega.is_contiguous()
    out = torch.empty_like(omega)
    s = lib.tdfe_power_spectrum(_ptr(mu), mu.numel(), float(dt), _ptr(omega), omega.numel(), _ptr(out),
                                _stream_handle())
    if s != OK:
        raise TdfeError(s, "power_spectrum: bad arguments")
    return out


def _adapt_desc(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples):
    keep = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1)) for v in (R, Z, s_orb, a_pot)]
    d = AdaptDesc()
    d.p, d.lo, d.hi, d.n_atoms = p, lo, hi, len(keep[1])
    d.R, d.Z, d.s_orb, d.a_pot = (k.ctypes.data_as(_DP) for k in keep)
    d.n_elem, d.samples = float(n_elem), samples
    return d, keep


def adaptive_axes(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples=129, max_cells=4096):
    """Vertex coordinates (x, y, z axes) of the graded rectilinear mesh whose
    spacing follows the a priori element size h(r); returns (axes, E)."""
    import torch
    lib = load()
    d, keep = _adapt_desc(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples)
    nb = ctypes.c_size_t()
    s = lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb))
    if s != OK:
        raise TdfeError(s, "adaptive_axes: bad description")
    scratch = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    base = scratch.data_ptr()
    off = (-base) % 256
    axes = np.zeros((3, max_cells + 1))
    nc = (ctypes.c_int * 3)()
    E = ctypes.c_double()
    s = lib.tdfe_adaptive_axes(ctypes.byref(d), ctypes.c_void_p(base + off), nb.value, _stream_handle(), max_cells,
                               axes.ctypes.data_as(_DP), nc, ctypes.byref(E))
    if s != OK:
        raise TdfeError(s, "adaptive_axes failed")
    del keep
    return [axes[a, :nc[a] + 1].copy() for a in range(3)], E.value


def octree_leaves(p, lo, hi, R, Z, s_orb, a_pot, n_elem, n0, max_level, samples=129, max_leaves=200000):
    """Leaves ({q, i, j, k} rows, sorted) of the balanced octree whose cubes
    follow the a priori element size h(r); returns (leaves, E)."""
    import torch
    lib = load()
    d, keep = _adapt_desc(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples)
    nb = ctypes.c_size_t()
    s = lib.tdfe_octree_leaves_query(ctypes.byref(d), max_leaves, ctypes.byref(nb))
    if s != OK:
        raise TdfeError(s, "octree_leaves: bad description")
    scratch = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    base = scratch.data_ptr()
    off = (-base) % 256
    out = np.zeros((max_leaves, 4), dtype=np.int32)
    n = ctypes.c_int()
    E = ctypes.c_double()
    s = lib.tdfe_octree_leaves(ctypes.byref(d), n0, max_level, ctypes.c_void_p(base + off), nb.value,
                               _stream_handle(), max_leaves, out.ctypes.data_as(_IP), ctypes.byref(n),
                               ctypes.byref(E))
    if s != OK:
        raise TdfeError(s, "octree_leaves failed")
    del keep
    return out[:n.value].copy(), E.value


def adaptive_axes_static(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples=129, max_cells=4096):
    """adaptive_axes through the allocation-free entry point (the library's own
    static device scratch; samples <= 160); returns (axes, E)."""
    lib = load()
    d, keep = _adapt_desc(p, lo, hi, R, Z, s_orb, a_pot, n_elem, samples)
    axes = np.zeros((3, max_cells + 1))
    nc = (ctypes.c_int * 3)()
    E = ctypes.c_double()
    s = lib.tdfe_adaptive_axes_static(ctypes.byref(d), _stream_handle(), max_cells, axes.ctypes.data_as(_DP), nc,
                                      ctypes.byref(E))
    if s != OK:
        raise TdfeError(s, "adaptive_axes_static failed")
    del keep
    return [axes[a, :nc[a] + 1].copy() for a in range(3)], E.value


def tridiag_expm(alpha, beta, tau):
    """y = exp(-i tau T) e_1 on the GPU for the tridiagonal T (numpy alpha[k],
    beta[k-1]); returns (y as a complex128 numpy array, number of series terms)."""
    import torch
    lib = load()
    k = len(alpha)
    nb = ctypes.c_size_t()
    s = lib.tdfe_tridiag_expm_query(k, ctypes.byref(nb))
    if s != OK:
        raise TdfeError(s, "tridiag_expm: bad order")
    a = torch.from_numpy(np.ascontiguousarray(alpha, dtype=np.float64)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))).cuda() if k > 1 else None
    y = torch.empty(k, dtype=torch.complex128, device="cuda")
    scratch = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    base = scratch.data_ptr()
    off = (-base) % 256
    m = ctypes.c_int()
    s = lib.tdfe_tridiag_expm(_ptr(a), _ptr(b) if b is not None else None, k, float(tau), _ptr(y),
                              ctypes.c_void_p(base + off), nb.value, _stream_handle(), ctypes.byref(m))
    if s != OK:
        raise TdfeError(s, "tridiag_expm failed")
    return y.cpu().numpy(), m.value


def rectilinear_vertices(ax, ay, az):
    """Vertex array [(nz+1)(ny+1)(nx+1)][3] (x fastest) of the tensor-product mesh."""
    Z3, Y3, X3 = np.meshgrid(az, ay, ax, indexing="ij")
    return np.stack([X3, Y3, Z3], axis=-1).reshape(-1, 3)
