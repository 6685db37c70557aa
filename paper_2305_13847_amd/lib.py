"""Thin ctypes binding of libdgmoist (include/dg.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the shared library.  Tensors are torch tensors on the GPU (torch supplies
memory and streams); shapes, dtypes and devices are checked here before any
pointer reaches the library.  There is no fallback: if the library is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmoist.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_ENOCONV, DG_ENONFINITE, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
DG_PERIODIC, DG_SLIPWALL = 0, 1
DG_FP64, DG_FP32_BULK = 0, 1
DG_SSPRK43, DG_SSPRK33 = 0, 1
DG_VR_CONST, DG_VR_COSMO = 0, 1
DG_BASIS_LOBATTO, DG_BASIS_GAUSS = 0, 1
BASES = {"lobatto": DG_BASIS_LOBATTO, "gauss": DG_BASIS_GAUSS}


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("dg status %d: %s" % (status, msg))
        self.status = status


class dg_mesh(ct.Structure):
    _fields_ = [("dim", ct.c_int), ("n", ct.c_int * 3), ("lo", ct.c_double * 3),
                ("hi", ct.c_double * 3), ("bc", ct.c_int * 3)]


class dg_params(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in
                ("g", "cvd", "cvv", "cl", "cpd", "cpv", "Rd", "Rv", "Lref", "Tref", "eref", "pref")] + \
               [("rain", ct.c_int), ("vr_mode", ct.c_int), ("vr_const", ct.c_double),
                ("rho_w", ct.c_double), ("N0r", ct.c_double), ("v0r", ct.c_double),
                ("q_au", ct.c_double), ("precision", ct.c_int), ("rk", ct.c_int),
                ("newton_rtol", ct.c_double), ("newton_maxit", ct.c_int),
                ("sponge_zD", ct.c_double), ("sponge_alpha", ct.c_double), ("basis", ct.c_int),
                ("sip_gamma", ct.c_double), ("sip_sigma", ct.c_double)]


class dg_tri_mesh(ct.Structure):
    _fields_ = [("ne", ct.c_int), ("xy", ct.POINTER(ct.c_double)), ("nb", ct.POINTER(ct.c_int)),
                ("nbf", ct.POINTER(ct.c_int)), ("z0", ct.c_double), ("dz", ct.c_double), ("nz", ct.c_int)]


class dg_stats(ct.Structure):
    _fields_ = [("splits", ct.c_longlong), ("nonconverged", ct.c_longlong),
                ("max_iters", ct.c_int), ("nonfinite", ct.c_int)]


EXPORTS = ["dg_default_params", "dg_create", "dg_create_batch", "dg_set_background",
           "dg_member_offset", "dg_state_size", "dg_rhs", "dg_saturation_split", "dg_rk_step",
           "dg_rhs_vjp", "dg_saturation_split_vjp", "dg_rk_step_vjp", "dg_reduce_mass", "dg_reduce_mass_member",
           "dg_get_stats", "dg_reset_stats", "dg_destroy", "dg_last_error", "dg_timing_enable",
           "dg_timing_read", "dg_set_launch", "dg_get_launch", "dg_autotune", "dg_rk_step_graph",
           "dg_rhs_noalloc", "dg_set_item_order", "dg_get_item_order",
           # triangles (include/dg_tri.h)
           "dg_tri_create", "dg_tri_set_background", "dg_tri_points", "dg_tri_state_size", "dg_tri_npoints",
           "dg_tri_project", "dg_tri_split", "dg_tri_rhs", "dg_tri_rk_step", "dg_tri_get_stats",
           "dg_tri_reset_stats", "dg_tri_timing_enable", "dg_tri_timing_read", "dg_tri_destroy"]
DG_K_SPLIT, DG_K_STAGE, DG_K_ADJOINT, DG_K_OTHER = 0, 1, 2, 3

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libdgmoist.so not built at %s (run __graft_entry__.build())" % path)
    L = ct.CDLL(path)
    vp, dp = ct.c_void_p, ct.POINTER(ct.c_double)
    L.dg_default_params.argtypes = [ct.POINTER(dg_params)]
    L.dg_default_params.restype = None
    L.dg_create.argtypes = [ct.POINTER(dg_mesh), ct.c_int, ct.c_int, ct.POINTER(dg_params), ct.POINTER(vp)]
    L.dg_create_batch.argtypes = [ct.POINTER(dg_mesh), ct.c_int, ct.c_int, ct.c_int, ct.POINTER(dg_params),
                                  ct.POINTER(vp)]
    L.dg_set_background.argtypes = [vp, dp, dp, dp, dp, ct.c_int]
    L.dg_member_offset.argtypes = [vp, ct.c_int, ct.POINTER(ct.c_longlong), ct.POINTER(ct.c_longlong)]
    L.dg_state_size.argtypes = [vp]
    L.dg_state_size.restype = ct.c_longlong
    L.dg_rhs.argtypes = [vp, vp, vp, vp]
    L.dg_rhs_noalloc.argtypes = [vp, vp, vp, vp]
    L.dg_saturation_split.argtypes = [vp, vp, vp, ct.c_int, vp, vp, vp]
    L.dg_rk_step.argtypes = [vp, vp, dp, ct.c_int, vp]
    L.dg_rhs_vjp.argtypes = [vp, vp, vp, vp, vp]
    L.dg_saturation_split_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.dg_rk_step_vjp.argtypes = [vp, vp, vp, vp, dp, vp]
    L.dg_reduce_mass.argtypes = [vp, vp, dp, vp]
    L.dg_reduce_mass_member.argtypes = [vp, vp, dp, ct.c_int, vp]
    L.dg_get_stats.argtypes = [vp, ct.POINTER(dg_stats)]
    L.dg_reset_stats.argtypes = [vp]
    L.dg_destroy.argtypes = [vp]
    L.dg_timing_enable.argtypes = [vp, ct.c_int]
    L.dg_timing_read.argtypes = [vp, ct.c_int, dp, ct.POINTER(ct.c_longlong)]
    L.dg_set_launch.argtypes = [vp, ct.c_int, ct.c_int]
    L.dg_get_launch.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
    L.dg_set_item_order.argtypes = [vp, ct.c_int]
    L.dg_get_item_order.argtypes = [vp, ct.POINTER(ct.c_int)]
    L.dg_autotune.argtypes = [vp, vp, dp, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), dp]
    L.dg_rk_step_graph.argtypes = [vp, vp, dp, ct.c_int, vp]
    L.dg_tri_create.argtypes = [ct.POINTER(dg_tri_mesh), ct.c_int, ct.c_int, ct.POINTER(dg_params), ct.POINTER(vp)]
    L.dg_tri_set_background.argtypes = [vp, dp, dp, dp, dp]
    L.dg_tri_points.argtypes = [vp, dp]
    L.dg_tri_state_size.argtypes = [vp]
    L.dg_tri_state_size.restype = ct.c_longlong
    L.dg_tri_npoints.argtypes = [vp]
    L.dg_tri_npoints.restype = ct.c_longlong
    L.dg_tri_project.argtypes = [vp, vp, ct.c_int, vp, vp]
    L.dg_tri_split.argtypes = [vp, vp, vp, vp, vp]
    L.dg_tri_rhs.argtypes = [vp, vp, vp, vp]
    L.dg_tri_rk_step.argtypes = [vp, vp, ct.c_double, ct.c_int, vp]
    L.dg_tri_get_stats.argtypes = [vp, ct.POINTER(dg_stats)]
    L.dg_tri_reset_stats.argtypes = [vp]
    L.dg_tri_timing_enable.argtypes = [vp, ct.c_int]
    L.dg_tri_timing_read.argtypes = [vp, ct.c_int, dp, ct.POINTER(ct.c_longlong)]
    L.dg_tri_destroy.argtypes = [vp]
    L.dg_last_error.argtypes = []
    L.dg_last_error.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("dg_default_params", "dg_state_size", "dg_last_error", "dg_tri_state_size",
                        "dg_tri_npoints"):
            getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def _check(status: int):
    if status != DG_OK:
        raise DGError(status, load().dg_last_error().decode())


def default_params(**over) -> dg_params:
    p = dg_params()
    load().dg_default_params(ct.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def make_mesh(dim, n, lo, hi, bc) -> dg_mesh:
    m = dg_mesh()
    m.dim = int(dim)
    for a in range(3):
        m.n[a] = int(n[a]) if a < dim else 1
        m.lo[a] = float(lo[a]) if a < dim else 0.0
        m.hi[a] = float(hi[a]) if a < dim else 1.0
        m.bc[a] = int(bc[a]) if a < dim else 0
    return m


def _stream(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class DG:
    """One handle: a mesh (or an ensemble of meshes), order, variables, model."""

    def __init__(self, meshes, order: int, nvars: int, params: dg_params):
        import torch
        self.L = load()
        if not isinstance(meshes, (list, tuple)):
            meshes = [meshes]
        arr = (dg_mesh * len(meshes))(*[make_mesh(m.dim, m.n, m.lo, m.hi, m.bc) for m in meshes])
        self.meshes, self.order, self.nvars, self.params = list(meshes), order, nvars, params
        self.dtype = torch.float64 if params.precision == DG_FP64 else torch.float32
        h = ct.c_void_p()
        _check(self.L.dg_create_batch(arr, len(meshes), order, nvars, ct.byref(params), ct.byref(h)))
        self.h = h
        self.size = int(self.L.dg_state_size(h))
        self.npe = (order + 1) ** meshes[0].dim
        self.nnodes = self.size // nvars
        self.offsets = []
        for m in range(len(meshes)):
            off, ne = ct.c_longlong(), ct.c_longlong()
            _check(self.L.dg_member_offset(h, m, ct.byref(off), ct.byref(ne)))
            self.offsets.append((off.value, ne.value))

    @property
    def shape(self):
        return (self.nvars, self.nnodes // self.npe, self.npe)

    def close(self):
        if getattr(self, "h", None):
            self.L.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks ---------------------------------------------------
    def _state(self, t, name="U"):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if t.dtype != self.dtype or not t.is_contiguous() or t.numel() != self.size:
            raise ValueError("%s must be a contiguous %s tensor with %d values" % (name, self.dtype, self.size))
        return ct.c_void_p(t.data_ptr())

    def _nodal(self, t, name):
        import torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
                or not t.is_contiguous() or t.numel() != self.nnodes:
            raise ValueError("%s must be a contiguous CUDA float64 tensor with %d values" % (name, self.nnodes))
        return ct.c_void_p(t.data_ptr())

    # -- calls ---------------------------------------------------------------
    def set_background(self, member: int, rho_d, rho_m, rho_r, E):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (rho_d, rho_m, E)]
        rr = None if rho_r is None else np.ascontiguousarray(rho_r, dtype=np.float64)
        dp = ct.POINTER(ct.c_double)
        m = self.meshes[member]
        nzq = m.n[m.dim - 1] * (self.order + 1)
        for x in a + ([rr] if rr is not None else []):
            if x.size != nzq:
                raise ValueError("background arrays need %d values" % nzq)
        _check(self.L.dg_set_background(self.h, a[0].ctypes.data_as(dp), a[1].ctypes.data_as(dp),
                                        None if rr is None else rr.ctypes.data_as(dp), a[2].ctypes.data_as(dp),
                                        int(member)))

    def rhs(self, U, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(U)
        _check(self.L.dg_rhs(self.h, self._state(U), self._state(out, "dUdt"), ct.c_void_p(_stream(stream))))
        return out

    def rhs_noalloc(self, U, out, stream=None):
        """dg_rhs with the split scratch in the library's static device array;
        `out` must be given (nothing is allocated)."""
        _check(self.L.dg_rhs_noalloc(self.h, self._state(U), self._state(out, "dUdt"), ct.c_void_p(_stream(stream))))
        return out

    def saturation_split(self, U, T=None, use_guess=False, stream=None):
        import torch
        dev = U.device
        if T is None:
            T = torch.empty(self.nnodes, dtype=torch.float64, device=dev)
        rv = torch.empty(self.nnodes, dtype=torch.float64, device=dev)
        rc = torch.empty(self.nnodes, dtype=torch.float64, device=dev)
        _check(self.L.dg_saturation_split(self.h, self._state(U), self._nodal(T, "T"), int(bool(use_guess)),
                                          self._nodal(rv, "rho_v"), self._nodal(rc, "rho_c"),
                                          ct.c_void_p(_stream(stream))))
        return T, rv, rc

    def rk_step(self, U, dt, nsteps: int = 1, stream=None):
        dts = np.ascontiguousarray(np.atleast_1d(np.asarray(dt, dtype=np.float64)))
        if dts.size != len(self.meshes):
            raise ValueError("dt needs %d values" % len(self.meshes))
        _check(self.L.dg_rk_step(self.h, self._state(U), dts.ctypes.data_as(ct.POINTER(ct.c_double)),
                                 int(nsteps), ct.c_void_p(_stream(stream))))
        return U

    def rk_step_graph(self, U, dt, nsteps: int = 1, stream=None):
        dts = np.ascontiguousarray(np.atleast_1d(np.asarray(dt, dtype=np.float64)))
        if dts.size != len(self.meshes):
            raise ValueError("dt needs %d values" % len(self.meshes))
        _check(self.L.dg_rk_step_graph(self.h, self._state(U), dts.ctypes.data_as(ct.POINTER(ct.c_double)),
                                       int(nsteps), ct.c_void_p(_stream(stream))))
        return U

    def set_launch(self, elems_per_block: int, persist_per_cu: int):
        _check(self.L.dg_set_launch(self.h, int(elems_per_block), int(persist_per_cu)))

    def get_launch(self):
        e, p = ct.c_int(), ct.c_int()
        _check(self.L.dg_get_launch(self.h, ct.byref(e), ct.byref(p)))
        return e.value, p.value

    def set_item_order(self, order: int):
        _check(self.L.dg_set_item_order(self.h, int(order)))

    def get_item_order(self) -> int:
        o = ct.c_int()
        _check(self.L.dg_get_item_order(self.h, ct.byref(o)))
        return o.value

    def autotune(self, U, dt, nsteps: int = 3, cache: Optional[str] = None, key: Optional[str] = None):
        """Pick elements per block and the persistent grid by timing; optional JSON cache."""
        import json
        if cache and key and os.path.exists(cache):
            with open(cache) as f:
                rec = json.load(f).get(key)
            if rec:
                self.set_item_order(rec.get("item_order", 0))
                self.set_launch(rec["elems_per_block"], rec["persist_per_cu"])
                return rec
        dts = np.ascontiguousarray(np.atleast_1d(np.asarray(dt, dtype=np.float64)))
        e, p, ms = ct.c_int(), ct.c_int(), ct.c_double()
        _check(self.L.dg_autotune(self.h, self._state(U), dts.ctypes.data_as(ct.POINTER(ct.c_double)),
                                  int(nsteps), ct.byref(e), ct.byref(p), ct.byref(ms)))
        rec = dict(elems_per_block=e.value, persist_per_cu=p.value, item_order=self.get_item_order(),
                   ms_per_step=ms.value)
        if cache and key:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = rec
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
        return rec

    def rhs_vjp(self, U, lam, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(U)
        _check(self.L.dg_rhs_vjp(self.h, self._state(U), self._state(lam, "dUdt_bar"),
                                 self._state(out, "U_bar"), ct.c_void_p(_stream(stream))))
        return out

    def saturation_split_vjp(self, U, T_bar=None, rho_v_bar=None, rho_c_bar=None, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(U)
        _check(self.L.dg_saturation_split_vjp(self.h, self._state(U), self._nodal(T_bar, "T_bar"),
                                              self._nodal(rho_v_bar, "rho_v_bar"),
                                              self._nodal(rho_c_bar, "rho_c_bar"), self._state(out, "U_bar"),
                                              ct.c_void_p(_stream(stream))))
        return out

    def rk_step_vjp(self, U_n, U_np1_bar, dt, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(U_n)
        dts = np.ascontiguousarray(np.atleast_1d(np.asarray(dt, dtype=np.float64)))
        if dts.size != len(self.meshes):
            raise ValueError("dt needs %d values" % len(self.meshes))
        _check(self.L.dg_rk_step_vjp(self.h, self._state(U_n), self._state(U_np1_bar, "U_np1_bar"),
                                     self._state(out, "U_n_bar"), dts.ctypes.data_as(ct.POINTER(ct.c_double)),
                                     ct.c_void_p(_stream(stream))))
        return out

    def reduce_mass(self, U, member: int = -1, stream=None):
        """(dry mass, total water, wall rain outflow) of all members, or of one."""
        out = np.zeros(3)
        o = out.ctypes.data_as(ct.POINTER(ct.c_double))
        if member < 0:
            _check(self.L.dg_reduce_mass(self.h, self._state(U), o, ct.c_void_p(_stream(stream))))
        else:
            _check(self.L.dg_reduce_mass_member(self.h, self._state(U), o, int(member),
                                                ct.c_void_p(_stream(stream))))
        return out

    def stats(self):
        s = dg_stats()
        st = self.L.dg_get_stats(self.h, ct.byref(s))
        return dict(status=st, splits=s.splits, nonconverged=s.nonconverged, max_iters=s.max_iters,
                    nonfinite=s.nonfinite)

    def timing(self, enable: bool = True):
        _check(self.L.dg_timing_enable(self.h, int(bool(enable))))

    def timing_read(self, kclass: int):
        ms, n = ct.c_double(), ct.c_longlong()
        _check(self.L.dg_timing_read(self.h, int(kclass), ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

    def reset_stats(self):
        _check(self.L.dg_reset_stats(self.h))


def params_for_case(case, precision=DG_FP64, **over) -> dg_params:
    over.setdefault("basis", BASES[getattr(case.mesh, "basis", "lobatto")])
    return default_params(g=case.g, rain=case.rain, vr_const=case.vr_const, precision=precision, **over)


def for_case(case, precision=DG_FP64, **over) -> DG:
    """Handle + background for a synthetic case (see synth.py)."""
    dg = DG(case.mesh, case.mesh.order, case.nvars, params_for_case(case, precision, **over))
    dg.set_background(0, case.bg["rho_d"], case.bg["rho_m"], case.bg["rho_r"], case.bg["E"])
    return dg


def for_ensemble(cases, precision=DG_FP32_BULK, **over) -> DG:
    c0 = cases[0]
    dg = DG([c.mesh for c in cases], c0.mesh.order, c0.nvars, params_for_case(c0, precision, **over))
    for m, c in enumerate(cases):
        dg.set_background(m, c.bg["rho_d"], c.bg["rho_m"], c.bg["rho_r"], c.bg["E"])
    return dg


class DGTri:
    """A triangulation handle (include/dg_tri.h): coefficients C[v][e][m]."""

    def __init__(self, mesh, nvars: int, params: dg_params):
        import torch
        self.L = load()
        self.mesh, self.nvars, self.params = mesh, nvars, params
        self.order = int(mesh.order)
        self.dtype = torch.float64 if params.precision == DG_FP64 else torch.float32
        self._xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        self._nb = np.ascontiguousarray(mesh.nb, dtype=np.int32)
        self._nbf = np.ascontiguousarray(mesh.nbf, dtype=np.int32)
        m = dg_tri_mesh()
        m.ne = int(mesh.ne)
        m.xy = self._xy.ctypes.data_as(ct.POINTER(ct.c_double))
        m.nb = self._nb.ctypes.data_as(ct.POINTER(ct.c_int))
        m.nbf = self._nbf.ctypes.data_as(ct.POINTER(ct.c_int))
        m.z0 = float(mesh.lo[1])
        m.dz = float(mesh.h[1])
        m.nz = int(mesh.n[1])
        h = ct.c_void_p()
        _check(self.L.dg_tri_create(ct.byref(m), self.order, nvars, ct.byref(params), ct.byref(h)))
        self.h = h
        self.size = int(self.L.dg_tri_state_size(h))
        self.npoints = int(self.L.dg_tri_npoints(h))
        self.np = (self.order + 1) * (self.order + 2) // 2
        self.nq = (self.order + 1) * (self.order + 2)
        self.ne = int(mesh.ne)

    @property
    def shape(self):
        return (self.nvars, self.ne, self.np)

    def close(self):
        if getattr(self, "h", None):
            self.L.dg_tri_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _coef(self, t, nfields, name="C"):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if t.dtype != self.dtype or not t.is_contiguous() or t.numel() != nfields * self.ne * self.np:
            raise ValueError("%s must be a contiguous %s tensor with %d values" % (name, self.dtype,
                                                                                  nfields * self.ne * self.np))
        return ct.c_void_p(t.data_ptr())

    def set_background(self, rho_d, rho_m, rho_r, E):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho_d, rho_m, rho_r, E)]
        n = int(self.mesh.n[1]) * (self.order + 1)
        if any(a.size != n for a in arrs):
            raise ValueError("background arrays need %d values" % n)
        self._bg = arrs
        dp = ct.POINTER(ct.c_double)
        _check(self.L.dg_tri_set_background(self.h, *[a.ctypes.data_as(dp) for a in arrs]))

    def points(self) -> np.ndarray:
        """Physical coordinates of the volume points, (ne, nq, 2)."""
        out = np.zeros((self.ne, self.nq, 2))
        _check(self.L.dg_tri_points(self.h, out.ctypes.data_as(ct.POINTER(ct.c_double))))
        return out

    def project(self, vals, stream=None):
        """Coefficients (nf, ne, np) of fields given at the volume points (nf, ne, nq), float64 on the GPU."""
        import torch
        if not isinstance(vals, torch.Tensor) or not vals.is_cuda or vals.dtype != torch.float64 \
                or not vals.is_contiguous() or vals.numel() % (self.ne * self.nq) != 0:
            raise ValueError("vals must be a contiguous CUDA float64 tensor of nf x ne x nq values")
        nf = vals.numel() // (self.ne * self.nq)
        out = torch.empty((nf, self.ne, self.np), dtype=self.dtype, device=vals.device)
        _check(self.L.dg_tri_project(self.h, ct.c_void_p(vals.data_ptr()), nf, ct.c_void_p(out.data_ptr()),
                                     ct.c_void_p(_stream(stream))))
        return out

    def state(self, point_state, device="cuda"):
        """Coefficients of a state given as a function of position (projected on the GPU)."""
        import torch
        vals = torch.from_numpy(np.ascontiguousarray(point_state(self.points()), dtype=np.float64)).to(device)
        return self.project(vals)

    def split(self, C, stream=None):
        """Coefficients (ne, np) of the projected T and rho_v."""
        import torch
        Tc = torch.empty((self.ne, self.np), dtype=torch.float64, device=C.device)
        Rc = torch.empty_like(Tc)
        _check(self.L.dg_tri_split(self.h, self._coef(C, self.nvars), ct.c_void_p(Tc.data_ptr()),
                                   ct.c_void_p(Rc.data_ptr()), ct.c_void_p(_stream(stream))))
        return Tc, Rc

    def rhs(self, C, out=None, stream=None):
        import torch
        out = torch.empty_like(C) if out is None else out
        _check(self.L.dg_tri_rhs(self.h, self._coef(C, self.nvars), self._coef(out, self.nvars, "out"),
                                 ct.c_void_p(_stream(stream))))
        return out

    def rk_step(self, C, dt: float, nsteps: int = 1, stream=None):
        _check(self.L.dg_tri_rk_step(self.h, self._coef(C, self.nvars), float(dt), int(nsteps),
                                     ct.c_void_p(_stream(stream))))
        return C

    def stats(self):
        s = dg_stats()
        st = self.L.dg_tri_get_stats(self.h, ct.byref(s))
        return dict(status=st, splits=s.splits, nonconverged=s.nonconverged, max_iters=s.max_iters,
                    nonfinite=s.nonfinite)

    def reset_stats(self):
        _check(self.L.dg_tri_reset_stats(self.h))

    def timing(self, enable: bool = True):
        _check(self.L.dg_tri_timing_enable(self.h, int(bool(enable))))

    def timing_read(self, kclass: int):
        ms, n = ct.c_double(), ct.c_longlong()
        _check(self.L.dg_tri_timing_read(self.h, int(kclass), ct.byref(ms), ct.byref(n)))
        return ms.value, n.value


def for_tri_case(case, precision=DG_FP64, **over) -> DGTri:
    """Triangulation handle + background for a synthetic triangle case (synth.tri_bubble)."""
    p = default_params(g=case.g, rain=case.rain, vr_const=case.vr_const, precision=precision, **over)
    dg = DGTri(case.mesh, case.nvars, p)
    dg.set_background(case.bg["rho_d"], case.bg["rho_m"], case.bg["rho_r"], case.bg["E"])
    return dg
