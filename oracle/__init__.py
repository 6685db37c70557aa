"""ctypes shim over the plain FP64 CPU reference (dg_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the library.  The reference shares no
source with the GPU path.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dg_oracle.cpp")
LIB = os.path.join(HERE, "libdgoracle.so")
# a prebuilt copy of the reference (the mutation checks load deliberately
# broken builds this way; it is never rebuilt from SRC)
LIB_OVERRIDE = os.environ.get("DG_ORACLE_LIB")


def build() -> str:
    """Compile the reference with -O2 and no fast-math; its element loops use
    OpenMP (the result does not depend on the thread count)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-fopenmp", "-o", LIB, SRC]
    subprocess.check_call(cmd)
    return LIB


class OraParams(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in
                ("g", "cvd", "cvv", "cl", "cpd", "cpv", "Rd", "Rv", "Lref", "Tref", "eref", "pref")] + \
               [("rain", ct.c_int), ("vr_mode", ct.c_int)] + \
               [(n, ct.c_double) for n in ("vr_const", "rho_w", "N0r", "v0r", "q_au", "sponge_zD", "sponge_alpha",
                                           "sip_gamma", "sip_sigma")]


class OraMesh(ct.Structure):
    _fields_ = [("dim", ct.c_int), ("n", ct.c_int * 3), ("lo", ct.c_double * 3),
                ("hi", ct.c_double * 3), ("bc", ct.c_int * 3), ("order", ct.c_int),
                ("basis", ct.c_int)]

BASES = {"lobatto": 0, "gauss": 1}


class OraTriMesh(ct.Structure):
    _fields_ = [("ne", ct.c_int), ("xy", ct.POINTER(ct.c_double)), ("nb", ct.POINTER(ct.c_int)),
                ("nbf", ct.POINTER(ct.c_int)), ("order", ct.c_int), ("z0", ct.c_double),
                ("dz", ct.c_double), ("nz", ct.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LIB_OVERRIDE:
            L = ct.CDLL(LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            L = ct.CDLL(LIB)
        dp = ct.POINTER(ct.c_double)
        L.ora_default_params.argtypes = [ct.POINTER(OraParams)]
        L.ora_tables.argtypes = [ct.c_int, dp, dp, dp, dp]
        L.ora_gauss_tables.argtypes = [ct.c_int, dp, dp]
        L.ora_project.argtypes = [ct.c_void_p, dp, dp]
        L.ora_sip.argtypes = [ct.c_void_p, dp, dp, dp]
        L.ora_sip_alpha.argtypes = [ct.c_void_p, dp, dp, dp]
        L.ora_set_threads.argtypes = [ct.c_int]
        L.ora_set_threads.restype = None
        L.ora_get_threads.argtypes = []
        L.ora_get_threads.restype = ct.c_int
        L.ora_esat.argtypes = [ct.POINTER(OraParams), ct.c_double]
        L.ora_esat.restype = ct.c_double
        L.ora_rho_vs.argtypes = [ct.POINTER(OraParams), ct.c_double]
        L.ora_rho_vs.restype = ct.c_double
        L.ora_split.argtypes = [ct.POINTER(OraParams)] + [ct.c_double] * 4 + [dp] * 3
        L.ora_split_jvp.argtypes = [ct.POINTER(OraParams)] + [ct.c_double] * 8 + [dp] * 4
        L.ora_create.argtypes = [ct.POINTER(OraMesh), ct.POINTER(OraParams), ct.c_int, dp, dp, dp, dp]
        L.ora_create.restype = ct.c_void_p
        L.ora_destroy.argtypes = [ct.c_void_p]
        L.ora_background_pressure.argtypes = [ct.c_void_p, dp]
        L.ora_split_field.argtypes = [ct.c_void_p, dp, dp, dp, dp, dp, dp]
        L.ora_rhs.argtypes = [ct.c_void_p, dp, dp, dp]
        L.ora_rk_step.argtypes = [ct.c_void_p, dp, ct.c_double, ct.c_int, ct.c_int, dp]
        L.ora_rhs_jvp.argtypes = [ct.c_void_p, dp, dp, dp, dp]
        L.ora_rk_jvp.argtypes = [ct.c_void_p, dp, dp, ct.c_double, ct.c_int, ct.c_int]
        L.ora_mass.argtypes = [ct.c_void_p, dp, dp]
        L.ora_sponge_delta.argtypes = [ct.c_void_p, ct.c_double]
        L.ora_sponge_delta.restype = ct.c_double
        L.ora_sponge_apply.argtypes = [ct.c_void_p, dp]
        L.ora_point.argtypes = [ct.c_void_p, dp, ct.c_int, dp, dp, dp]
        L.ora_face.argtypes = [ct.c_void_p, dp, ct.c_int, dp, ct.c_int, ct.c_int, dp]
        L.ora_stats.argtypes = [ct.c_void_p, ct.POINTER(ct.c_long), ct.POINTER(ct.c_int),
                                ct.POINTER(ct.c_int)]
        ip = ct.POINTER(ct.c_int)
        L.ora_tri_rule.argtypes = [ct.c_int, dp, dp]
        L.ora_tri_basis.argtypes = [ct.c_int, dp, ct.c_int, dp, dp, dp]
        L.ora_tri_create.argtypes = [ct.POINTER(OraTriMesh), ct.POINTER(OraParams), ct.c_int, dp, dp, dp, dp]
        L.ora_tri_create.restype = ct.c_void_p
        L.ora_tri_destroy.argtypes = [ct.c_void_p]
        L.ora_tri_points.argtypes = [ct.c_void_p, dp]
        L.ora_tri_project.argtypes = [ct.c_void_p, dp, ct.c_int, dp]
        L.ora_tri_eval.argtypes = [ct.c_void_p, dp, ct.c_int, dp, ct.c_int, dp]
        L.ora_tri_background.argtypes = [ct.c_void_p, ct.c_double, dp]
        L.ora_tri_split.argtypes = [ct.c_void_p, dp, dp, dp]
        L.ora_tri_rhs.argtypes = [ct.c_void_p, dp, dp, dp]
        L.ora_tri_rk_step.argtypes = [ct.c_void_p, dp, ct.c_double, ct.c_int, ct.c_int, dp]
        L.ora_tri_mass.argtypes = [ct.c_void_p, dp, dp]
        L.ora_tri_face.argtypes = [ct.c_void_p, dp, dp, ct.c_double, dp, dp]
        L.ora_tri_stats.argtypes = [ct.c_void_p, ct.POINTER(ct.c_long), ct.POINTER(ct.c_int), ip]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def default_params(**over) -> OraParams:
    p = OraParams()
    lib().ora_default_params(ct.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def tables(k: int):
    p1 = k + 1
    x, w = np.zeros(p1), np.zeros(p1)
    D, Dh = np.zeros((p1, p1)), np.zeros((p1, p1))
    rc = lib().ora_tables(k, _p(x), _p(w), _p(D), _p(Dh))
    assert rc == 0
    return x, w, D, Dh


def gauss_tables(k: int):
    """The (k+1)-point Gauss-Legendre rule of the modal basis: points, weights."""
    x, w = np.zeros(k + 1), np.zeros(k + 1)
    if lib().ora_gauss_tables(k, _p(x), _p(w)) != 0:
        raise ValueError("order out of range")
    return x, w


def esat(P: OraParams, T: float) -> float:
    return lib().ora_esat(ct.byref(P), T)


def rho_vs(P: OraParams, T: float) -> float:
    return lib().ora_rho_vs(ct.byref(P), T)


def split(P: OraParams, rd, rm, rr, re):
    T, rv, rc = ct.c_double(), ct.c_double(), ct.c_double()
    it = lib().ora_split(ct.byref(P), rd, rm, rr, re, ct.byref(T), ct.byref(rv), ct.byref(rc))
    return T.value, rv.value, rc.value, it


def split_jvp(P: OraParams, x, dx):
    T, dT, rv, drv = (ct.c_double() for _ in range(4))
    rc = lib().ora_split_jvp(ct.byref(P), *x, *dx, ct.byref(T), ct.byref(dT), ct.byref(rv),
                             ct.byref(drv))
    assert rc == 0
    return T.value, dT.value, rv.value, drv.value


class Oracle:
    """One mesh + background; all arrays float64 in the U[v][e][n] layout."""

    def __init__(self, mesh, params: OraParams, nvars: int, bg: Dict[str, np.ndarray]):
        M = OraMesh()
        M.dim = mesh.dim
        for a in range(mesh.dim):
            M.n[a] = int(mesh.n[a]); M.lo[a] = float(mesh.lo[a]); M.hi[a] = float(mesh.hi[a])
            M.bc[a] = int(mesh.bc[a])
        M.order = mesh.order
        M.basis = BASES[getattr(mesh, "basis", "lobatto")]
        self.mesh, self.P, self.nvars = mesh, params, nvars
        self._bg = [np.ascontiguousarray(bg[k], dtype=np.float64) for k in ("rho_d", "rho_m", "rho_r", "E")]
        self.h = lib().ora_create(ct.byref(M), ct.byref(params), nvars, *[_p(a) for a in self._bg])
        if not self.h:
            raise ValueError("oracle rejected the mesh/order/nvars")
        self.shape = (nvars, mesh.ne, mesh.npe)

    @classmethod
    def for_case(cls, case, **over):
        P = default_params(g=case.g, rain=case.rain, vr_const=case.vr_const, **over)
        return cls(case.mesh, P, case.nvars, case.bg)

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "h", None) and lib is not None:
            try:
                lib().ora_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def pbar(self) -> np.ndarray:
        out = np.zeros(self.mesh.nzq)
        lib().ora_background_pressure(self.h, _p(out))
        return out

    def split_field(self, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        outs = [np.zeros(self.shape[1:]) for _ in range(5)]
        bad = lib().ora_split_field(self.h, _p(U), *[_p(o) for o in outs])
        return dict(T=outs[0], rho_v=outs[1], rho_c=outs[2], p_prime=outs[3], c_m=outs[4], bad=bad)

    def rhs(self, U: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.zeros_like(U)
        f = ct.c_double()
        lib().ora_rhs(self.h, _p(U), _p(dU), ct.byref(f))
        return dU

    def rk(self, U: np.ndarray, dt: float, nsteps: int, scheme: int = 0):
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        f = ct.c_double()
        lib().ora_rk_step(self.h, _p(U), dt, nsteps, scheme, ct.byref(f))
        return U, f.value

    def rhs_jvp(self, U: np.ndarray, V: np.ndarray):
        U = np.ascontiguousarray(U, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        dU, JV = np.zeros_like(U), np.zeros_like(U)
        lib().ora_rhs_jvp(self.h, _p(U), _p(V), _p(dU), _p(JV))
        return dU, JV

    def rk_jvp(self, U: np.ndarray, V: np.ndarray, dt: float, nsteps: int, scheme: int = 0):
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        V = np.array(V, dtype=np.float64, order="C", copy=True)
        lib().ora_rk_jvp(self.h, _p(U), _p(V), dt, nsteps, scheme)
        return U, V

    def mass(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(3)
        lib().ora_mass(self.h, _p(U), _p(out))
        return out

    def sponge_delta(self, z: float) -> float:
        """Blending function of the sponge layer at height z."""
        return lib().ora_sponge_delta(self.h, float(z))

    def sponge(self, U: np.ndarray) -> np.ndarray:
        """The end-of-step sponge applied once to a copy of U."""
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        lib().ora_sponge_apply(self.h, _p(U))
        return U

    def point(self, Uq: np.ndarray, iz: int):
        Uq = np.ascontiguousarray(Uq, dtype=np.float64)
        d = self.mesh.dim
        F, G, lam = np.zeros((d, self.nvars)), np.zeros(self.nvars), np.zeros(d)
        lib().ora_point(self.h, _p(Uq), iz, _p(F), _p(G), _p(lam))
        return F, G, lam

    def face(self, Um: np.ndarray, izm: int, Up: np.ndarray, izp: int, j: int):
        Um = np.ascontiguousarray(Um, dtype=np.float64)
        Up = np.ascontiguousarray(Up, dtype=np.float64)
        Fs = np.zeros(self.nvars)
        lib().ora_face(self.h, _p(Um), izm, _p(Up), izp, j, _p(Fs))
        return Fs

    def sip(self, U: np.ndarray, W: Optional[np.ndarray] = None) -> np.ndarray:
        """-M^{-1} A_h(U, .), the artificial diffusion alone, with the viscosity of W's velocity
        (W = U if not given)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        W = U if W is None else np.ascontiguousarray(W, dtype=np.float64)
        out = np.zeros_like(U)
        if lib().ora_sip(self.h, _p(U), _p(W), _p(out)) != 0:
            raise ValueError("needs the Lobatto basis and sip_gamma > 0")
        return out

    def sip_alpha(self, W: np.ndarray):
        """Nodal viscosity (every variable but rho_r, and rho_r) from W's velocity."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        a0 = np.zeros(W.shape[1:])
        a1 = np.zeros(W.shape[1:])
        if lib().ora_sip_alpha(self.h, _p(W), _p(a0), _p(a1)) != 0:
            raise ValueError("needs the Lobatto basis and sip_gamma > 0")
        return a0, a1

    def project(self, U: np.ndarray) -> np.ndarray:
        """Legendre coefficients of a state given at the Gauss points (modal basis)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        C = np.zeros_like(U)
        if lib().ora_project(self.h, _p(U), _p(C)) != 0:
            raise ValueError("projection needs the modal (gauss) basis")
        return C

    def stats(self):
        it, mx, bad = ct.c_long(), ct.c_int(), ct.c_int()
        lib().ora_stats(self.h, ct.byref(it), ct.byref(mx), ct.byref(bad))
        return dict(iters_total=it.value, max_iters=mx.value, bad=bad.value)


def set_threads(n: int) -> None:
    """Threads of the reference's element loops (n < 1: all cores)."""
    lib().ora_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ora_get_threads())


# ----------------------------------------------------------------------------
# triangles
# ----------------------------------------------------------------------------
def tri_rule(k: int):
    """The unit-triangle volume rule: points (n, 2) as (r, s) and weights (n,)."""
    n = (k + 1) * (k + 2)
    rs, w = np.zeros((n, 2)), np.zeros(n)
    if lib().ora_tri_rule(k, _p(rs), _p(w)) != n:
        raise ValueError("order out of range")
    return rs, w


def tri_basis(k: int, rs: np.ndarray):
    """Orthonormal basis and its reference gradient at points rs (n, 2):
    arrays (n, np) of psi, d/dr, d/ds."""
    rs = np.ascontiguousarray(rs, dtype=np.float64).reshape(-1, 2)
    npk = (k + 1) * (k + 2) // 2
    psi, dr, ds = (np.zeros((rs.shape[0], npk)) for _ in range(3))
    if lib().ora_tri_basis(k, _p(rs), rs.shape[0], _p(psi), _p(dr), _p(ds)) != npk:
        raise ValueError("order out of range")
    return psi, dr, ds


class TriOracle:
    """One triangulation + background; coefficients C[v][e][m] in float64."""

    def __init__(self, mesh, params: OraParams, nvars: int, bg: Dict[str, np.ndarray]):
        self.mesh, self.P, self.nvars = mesh, params, nvars
        self._xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        self._nb = np.ascontiguousarray(mesh.nb, dtype=np.int32)
        self._nbf = np.ascontiguousarray(mesh.nbf, dtype=np.int32)
        M = OraTriMesh()
        M.ne = mesh.ne
        M.xy = _p(self._xy)
        M.nb = self._nb.ctypes.data_as(ct.POINTER(ct.c_int))
        M.nbf = self._nbf.ctypes.data_as(ct.POINTER(ct.c_int))
        M.order = mesh.order
        M.z0 = float(mesh.lo[1])
        M.dz = float(mesh.h[1])
        M.nz = int(mesh.n[1])
        self._bg = [np.ascontiguousarray(bg[k], dtype=np.float64) for k in ("rho_d", "rho_m", "rho_r", "E")]
        self.h = lib().ora_tri_create(ct.byref(M), ct.byref(params), nvars, *[_p(a) for a in self._bg])
        if not self.h:
            raise ValueError("oracle rejected the triangulation/order/nvars")
        self.k = mesh.order
        self.np = (self.k + 1) * (self.k + 2) // 2
        self.nq = (self.k + 1) * (self.k + 2)
        self.shape = (nvars, mesh.ne, self.np)

    @classmethod
    def for_case(cls, case, **over):
        P = default_params(g=case.g, rain=case.rain, vr_const=case.vr_const, **over)
        return cls(case.mesh, P, case.nvars, case.bg)

    def __del__(self):
        if getattr(self, "h", None) and lib is not None:
            try:
                lib().ora_tri_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def points(self) -> np.ndarray:
        """Physical coordinates of the volume points, (ne, nq, 2)."""
        out = np.zeros((self.mesh.ne, self.nq, 2))
        lib().ora_tri_points(self.h, _p(out))
        return out

    def project(self, vals: np.ndarray) -> np.ndarray:
        """Coefficients of fields given at the volume points, (nf, ne, nq) -> (nf, ne, np)."""
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        nf = vals.shape[0]
        C = np.zeros((nf, self.mesh.ne, self.np))
        lib().ora_tri_project(self.h, _p(vals), nf, _p(C))
        return C

    def state(self, point_state) -> np.ndarray:
        """Coefficients of a state given as a function of position."""
        return self.project(point_state(self.points()))

    def eval(self, C: np.ndarray, rs: np.ndarray) -> np.ndarray:
        """Fields C (nf, ne, np) at reference points rs (n, 2): (nf, ne, n)."""
        C = np.ascontiguousarray(C, dtype=np.float64)
        rs = np.ascontiguousarray(rs, dtype=np.float64).reshape(-1, 2)
        out = np.zeros((C.shape[0], self.mesh.ne, rs.shape[0]))
        lib().ora_tri_eval(self.h, _p(C), C.shape[0], _p(rs), rs.shape[0], _p(out))
        return out

    def background(self, z: float) -> np.ndarray:
        out = np.zeros(5)
        lib().ora_tri_background(self.h, float(z), _p(out))
        return out

    def split(self, C: np.ndarray):
        """Coefficients of the projected T and rho_v, and the count of failed splits."""
        C = np.ascontiguousarray(C, dtype=np.float64)
        Tc, Rc = np.zeros(self.shape[1:]), np.zeros(self.shape[1:])
        bad = lib().ora_tri_split(self.h, _p(C), _p(Tc), _p(Rc))
        return Tc, Rc, bad

    def rhs(self, C: np.ndarray, with_flux: bool = False):
        C = np.ascontiguousarray(C, dtype=np.float64)
        dC = np.zeros_like(C)
        f = ct.c_double()
        lib().ora_tri_rhs(self.h, _p(C), _p(dC), ct.byref(f))
        return (dC, f.value) if with_flux else dC

    def rk(self, C: np.ndarray, dt: float, nsteps: int, scheme: int = 0):
        C = np.array(C, dtype=np.float64, order="C", copy=True)
        f = ct.c_double()
        lib().ora_tri_rk_step(self.h, _p(C), dt, nsteps, scheme, ct.byref(f))
        return C, f.value

    def mass(self, C: np.ndarray) -> np.ndarray:
        C = np.ascontiguousarray(C, dtype=np.float64)
        out = np.zeros(3)
        lib().ora_tri_mass(self.h, _p(C), _p(out))
        return out

    def face(self, Um: np.ndarray, Up: np.ndarray, z: float, n) -> np.ndarray:
        """Lax-Friedrichs flux along the unit normal n between two states at height z."""
        Um = np.ascontiguousarray(Um, dtype=np.float64)
        Up = np.ascontiguousarray(Up, dtype=np.float64)
        nn = np.ascontiguousarray(n, dtype=np.float64)
        Fs = np.zeros(self.nvars)
        lib().ora_tri_face(self.h, _p(Um), _p(Up), float(z), _p(nn), _p(Fs))
        return Fs

    def stats(self):
        it, mx, bad = ct.c_long(), ct.c_int(), ct.c_int()
        lib().ora_tri_stats(self.h, ct.byref(it), ct.byref(mx), ct.byref(bad))
        return dict(iters_total=it.value, max_iters=mx.value, bad=bad.value)
