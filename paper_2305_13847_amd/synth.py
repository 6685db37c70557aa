"""Seeded synthetic inputs for the moist DG hot path.

This module builds the arrays that both the HIP library and the CPU checker
receive: mesh descriptions, hydrostatic-like background profiles at the node
heights, and perturbation states in the library's ``U[v][e][n]`` layout.  It
holds no part of the discretisation itself (no saturation inversion, no flux,
no quadrature weights, no time stepping).  States are *constructed* from a
temperature and a water partition; the partition uses the Magnus-type fit of
the saturation vapour pressure (Alduchov & Eskridge 1996), deliberately not the
Clausius-Clapeyron form of the paper, so that whichever side inverts the state
later does so with its own saturation law.  The one exception is the
saturated gravity-wave state, built with the paper's law (see paper_rho_vs).
The conserved energy is then the paper's definition of E (Section 2,
energy-temperature relation).

Shapes follow the paper's workloads: the rising moist bubble (Section 4.2,
Appendix B.2), the warm-rain thermals (Sections 4.5-4.6) and smooth periodic
fields for small parity cases.  Every random number comes from numpy's PCG64
with a recorded seed.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

# Thermodynamic constants as printed in the paper's appendix table; g is not in
# that table and is the usual 9.81 m s^-2.
C = dict(cl=4218.0, cpd=1005.0, cpv=1850.0, cvd=718.0, cvv=1390.0,
         eref=610.7, Lref=2.835e6, Rd=287.05, Rv=461.51, Tref=273.15,
         pref=1.0e5, g=9.81)

PERIODIC, WALL = 0, 1
C_BOUND = 350.0   # upper bound on the sound speed used for the time step


@dataclasses.dataclass
class Mesh:
    """Structured box of ``n`` elements per axis; the last axis is vertical."""
    dim: int
    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc: Sequence[int]
    order: int
    # "lobatto": nodes at the Gauss-Lobatto points (collocation); "gauss":
    # nodes at the Gauss-Legendre points (the paper's modal Legendre space
    # with Gauss quadrature, held by its values at the quadrature points)
    basis: str = "lobatto"

    @property
    def ne(self) -> int:
        return int(np.prod(self.n))

    @property
    def npe(self) -> int:
        return (self.order + 1) ** self.dim

    @property
    def h(self) -> np.ndarray:
        return (np.asarray(self.hi, float) - np.asarray(self.lo, float)) / np.asarray(self.n, float)

    @property
    def nzq(self) -> int:
        """Number of distinct node heights (vertical elements x nodes per line)."""
        return self.n[-1] * (self.order + 1)


@dataclasses.dataclass
class Case:
    name: str
    mesh: Mesh
    nvars: int
    rain: int
    g: float
    vr_const: float
    bg: Dict[str, np.ndarray]         # rho_d, rho_m, rho_r, E at node heights
    U: np.ndarray                     # (nvars, ne, npe) float64 perturbation state
    dt: float
    nsteps: int
    seed: int
    info: Dict[str, float] = dataclasses.field(default_factory=dict)
    bg_full: Optional[Dict[str, np.ndarray]] = None   # adds T and p of the construction

    def digest(self) -> str:
        h = hashlib.sha256()
        for k in ("rho_d", "rho_m", "rho_r", "E"):
            h.update(np.ascontiguousarray(self.bg[k]).tobytes())
        h.update(np.ascontiguousarray(self.U).tobytes())
        return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def _sfx(basis: str) -> str:
    return "" if basis == "lobatto" else "-" + basis


def lobatto_points(k: int) -> np.ndarray:
    """Gauss-Lobatto points on [-1, 1]: +-1 and the roots of P_k' (numpy)."""
    from numpy.polynomial import legendre as L
    if k == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(k + 1)
    c[-1] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(c))))
    return np.concatenate([[-1.0], inner, [1.0]])


def gauss_points(k: int) -> np.ndarray:
    """The k + 1 Gauss-Legendre points on [-1, 1] (numpy)."""
    return np.polynomial.legendre.leggauss(k + 1)[0]


def mesh_points(mesh: Mesh) -> np.ndarray:
    """Reference node positions of the mesh's basis."""
    if mesh.basis == "gauss":
        return gauss_points(mesh.order)
    if mesh.basis != "lobatto":
        raise ValueError("unknown basis %r" % (mesh.basis,))
    return lobatto_points(mesh.order)


def node_coords(mesh: Mesh) -> List[np.ndarray]:
    """Physical coordinates of every node, one (ne, npe) array per axis."""
    k, d = mesh.order, mesh.dim
    xi = mesh_points(mesh)
    p1 = k + 1
    # element multi-index (x fastest) and node multi-index (i fastest)
    e_idx = np.unravel_index(np.arange(mesh.ne), tuple(reversed(mesh.n)))
    e_idx = list(reversed(e_idx))                   # e_idx[a] = element index along axis a
    n_idx = np.unravel_index(np.arange(p1 ** d), (p1,) * d)
    n_idx = list(reversed(n_idx))                   # n_idx[a] = node index along axis a
    h = mesh.h
    out = []
    for a in range(d):
        x = (mesh.lo[a] + (e_idx[a][:, None] + 0.5 * (xi[n_idx[a]][None, :] + 1.0)) * h[a])
        out.append(x)
    return out


def node_heights(mesh: Mesh) -> np.ndarray:
    """Height of every vertical node index iz = ez*(k+1) + l."""
    xi = mesh_points(mesh)
    hz = mesh.h[-1]
    ez = np.arange(mesh.n[-1])
    z = mesh.lo[-1] + (ez[:, None] + 0.5 * (xi[None, :] + 1.0)) * hz
    return z.reshape(-1)


def height_index(mesh: Mesh) -> np.ndarray:
    """(ne, npe) map from a node to its vertical index iz."""
    p1 = mesh.order + 1
    ez = np.arange(mesh.ne) // int(np.prod(mesh.n[:-1]))
    l = np.arange(p1 ** mesh.dim) // (p1 ** (mesh.dim - 1))
    return ez[:, None] * p1 + l[None, :]


# ----------------------------------------------------------------------------
# state construction
# ----------------------------------------------------------------------------
def magnus_rho_vs(T):
    """Approximate saturation vapour density, Magnus fit over liquid water."""
    es = 610.94 * np.exp(17.625 * (T - 273.15) / (T - 30.11))
    return es / (C["Rv"] * T)


def paper_rho_vs(T):
    """Saturation vapour density of the paper's Clausius-Clapeyron law (Section 2.1).

    Only the gravity-wave set-up uses it: that initial state is saturated
    throughout and its recipe (Appendix B.1) is stated in the paper's own law.
    Built with another law, the saturated base state is slightly out of
    balance for the solver, and the case's convergence stalls near h^1.5.
    """
    a = (C["cpv"] - C["cl"]) / C["Rv"]
    b = (C["Lref"] - (C["cpv"] - C["cl"]) * C["Tref"]) / C["Rv"]
    es = C["eref"] * (T / C["Tref"]) ** a * np.exp(b * (1.0 / C["Tref"] - 1.0 / T))
    return es / (C["Rv"] * T)


def energy(rho_d, rho_v, rho_c, rho_r, T, m2_over_rho=0.0):
    """Paper's total energy density for a given temperature and partition."""
    Cv = C["cvd"] * rho_d + C["cvv"] * rho_v + C["cl"] * (rho_c + rho_r)
    return Cv * (T - C["Tref"]) + rho_v * (C["Lref"] - C["Rv"] * C["Tref"]) + 0.5 * m2_over_rho


def energy_dT(rho_d, rho_m, rho_r, T):
    """d energy / dT at fixed densities, with the Magnus partition."""
    rvs = magnus_rho_vs(T)
    sat = rho_m > rvs
    Cv = np.where(sat, C["cvd"] * rho_d + C["cvv"] * rvs + C["cl"] * (rho_m - rvs + rho_r),
                  C["cvd"] * rho_d + C["cvv"] * rho_m + C["cl"] * rho_r)
    # d rvs/dT of the Magnus fit
    a, b = 17.625, 30.11
    dlnes = a * (273.15 - b) / (T - b) ** 2
    drvs = rvs * (dlnes - 1.0 / T)
    Leff = (C["cvv"] - C["cl"]) * (T - C["Tref"]) + C["Lref"] - C["Rv"] * C["Tref"]
    return Cv + np.where(sat, drvs * Leff, 0.0)


def partitioned_energy(rho_d, rho_m, rho_r, T, m2_over_rho=0.0):
    rvs = magnus_rho_vs(T)
    rho_v = np.minimum(rho_m, rvs)
    return energy(rho_d, rho_v, rho_m - rho_v, rho_r, T, m2_over_rho)


def background(mesh: Mesh, Ts: float, ratio: Callable[[np.ndarray], np.ndarray],
               lapse: float = 6.5e-3, p0: float = 1.0e5, g: float = 9.81) -> Dict[str, np.ndarray]:
    """Hydrostatic-like background at node heights.

    T(z) = Ts - lapse*z, rho_m = ratio(z) * rho_vs(T) with the Magnus fit, and
    dp/dz = -g (rho_d + rho_m) integrated from p(0) = p0.  Only the arrays the
    library consumes are returned (rho_d, rho_m, rho_r, E); the pressure is
    reconstructed by each solver from these.
    """
    return background_at(node_heights(mesh), Ts, ratio, lapse, p0, g)


def background_at(z, Ts: float, ratio: Callable[[np.ndarray], np.ndarray], lapse: float = 6.5e-3,
                  p0: float = 1.0e5, g: float = 9.81) -> Dict[str, np.ndarray]:
    """The profile of ``background`` at arbitrary heights z (any shape)."""
    from scipy.integrate import solve_ivp
    z = np.asarray(z, dtype=np.float64)

    def parts(zz, p):
        T = Ts - lapse * zz
        rvs = magnus_rho_vs(T)
        rm = ratio(np.asarray(zz)) * rvs
        rv = np.minimum(rm, rvs)
        rd = (p / T - C["Rv"] * rv) / C["Rd"]
        return T, rd, rm, rv

    def rhs(zz, p):
        _, rd, rm, _ = parts(zz, p)
        return -g * (rd + rm)

    zs = np.unique(np.concatenate([[0.0], z.ravel()]))
    sol = solve_ivp(rhs, (0.0, float(zs[-1])), [p0], t_eval=zs, rtol=1e-12, atol=1e-9,
                    method="DOP853")
    p = np.interp(z, sol.t, sol.y[0])
    T, rd, rm, rv = parts(z, p)
    rc = rm - rv
    E = energy(rd, rv, rc, 0.0, T)
    return dict(rho_d=rd, rho_m=rm, rho_r=np.zeros_like(z), E=E, T=T, p=p)


def bubble(X: List[np.ndarray], centre, radius, amp) -> np.ndarray:
    """cos^2 bubble of the rising-thermal set-ups (Appendix B.2 shape)."""
    L2 = sum(((X[a] - centre[a]) / radius) ** 2 for a in range(len(X)))
    L = np.minimum(np.sqrt(L2), 1.0)
    return amp * np.cos(0.5 * np.pi * L) ** 2


def cfl_dt(mesh: Mesh, umax: float, vr: float, cfl: float) -> float:
    k = mesh.order
    return float(cfl * np.min(mesh.h) / ((2 * k + 1) * (C_BOUND + umax + vr)))


def _layout(fields: List[np.ndarray]) -> np.ndarray:
    return np.ascontiguousarray(np.stack(fields, axis=0), dtype=np.float64)


def _bg_at_nodes(mesh: Mesh, bg: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    iz = height_index(mesh)
    return {k: v[iz] for k, v in bg.items()}


def theta_to_state(mesh: Mesh, bg: Dict[str, np.ndarray], theta: np.ndarray,
                   rain: bool) -> np.ndarray:
    """Perturbation state for a potential-temperature perturbation at rest.

    rho_d' = rho_m' = 0, m = 0 and E' = E(T_bg + T') - E_bg with
    T' = theta' (p_bg/p_ref)^(R_d/c_pd).
    """
    b = _bg_at_nodes(mesh, bg)
    Tp = theta * (b["p"] / C["pref"]) ** (C["Rd"] / C["cpd"])
    E1 = partitioned_energy(b["rho_d"], b["rho_m"], b["rho_r"], b["T"] + Tp)
    E0 = partitioned_energy(b["rho_d"], b["rho_m"], b["rho_r"], b["T"])
    z = np.zeros_like(theta)
    flds = [z, z.copy()] + ([z.copy()] if rain else []) + [z.copy() for _ in range(mesh.dim)] + [E1 - E0]
    return _layout(flds)


def theta_to_state_jvp(mesh: Mesh, bg: Dict[str, np.ndarray], theta: np.ndarray) -> np.ndarray:
    """d E'/d theta' per node (the only component of U that depends on theta')."""
    b = _bg_at_nodes(mesh, bg)
    ex = (b["p"] / C["pref"]) ** (C["Rd"] / C["cpd"])
    return energy_dT(b["rho_d"], b["rho_m"], b["rho_r"], b["T"] + theta * ex) * ex


def add_noise(rng: np.random.Generator, U: np.ndarray, mesh: Mesh, b: Dict[str, np.ndarray],
              rain: bool, level: float = 1e-4) -> None:
    rho = b["rho_d"] + b["rho_m"]
    scales = [b["rho_d"], b["rho_m"]] + ([1e-3 * np.ones_like(rho)] if rain else []) \
        + [rho * 1.0] * mesh.dim + [b["E"]]
    for v, s in enumerate(scales):
        U[v] += level * s * rng.standard_normal(U[v].shape)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
def _modes(rng, X, L, nmodes=3):
    """Normalised sum of smooth periodic modes with integer wave vectors."""
    s = np.zeros_like(X[0])
    for _ in range(nmodes):
        kv = rng.integers(1, 4, size=len(X))
        w = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2 * np.pi)
        s += w * np.sin(sum(2 * np.pi * kv[a] * X[a] / L[a] for a in range(len(X))) + ph)
    return s / np.max(np.abs(s))


def periodic_smooth(n=(16, 16), order=2, seed=1, nsteps=10, sat_fraction=0.3,
                    dim=2, basis="lobatto") -> Case:
    """Smooth periodic moist fields on the unit square (or cube), g = 0.

    Densities vary by 1%, the moist mixing ratio spans 2-20 g/kg, the velocity
    is 1% of a 340 m/s sound speed, and the all-vapour temperature is shifted so
    that about ``sat_fraction`` of the nodes are supersaturated before the
    split (by the Magnus estimate).
    """
    rng = np.random.default_rng(seed)
    mesh = Mesh(dim, list(n), [0.0] * dim, [1.0] * dim, [PERIODIC] * dim, order, basis)
    X = node_coords(mesh)
    Ls = [1.0] * dim
    s_d, s_q, s_T = (_modes(rng, X, Ls) for _ in range(3))
    s_u = [_modes(rng, X, Ls) for _ in range(dim)]
    rd = 1.16 * (1.0 + 1e-2 * s_d)
    qm = 2e-3 + 18e-3 * (s_q - s_q.min()) / (s_q.max() - s_q.min())
    rm = qm * rd
    rho = rd + rm
    u = [1e-2 * 340.0 * su for su in s_u]
    m = [rho * ua for ua in u]
    m2r = sum(ma * ma for ma in m) / rho

    def frac_sat(T0):
        Tu = T0 * (1.0 + 1e-2 * s_T)
        return float(np.mean(rm > magnus_rho_vs(Tu)))

    lo, hi = 250.0, 330.0           # frac_sat decreases with T0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if frac_sat(mid) > sat_fraction:
            lo = mid
        else:
            hi = mid
    T0 = 0.5 * (lo + hi)
    Tu = T0 * (1.0 + 1e-2 * s_T)
    E = energy(rd, rm, 0.0, 0.0, Tu, m2r)     # all water counted as vapour
    bg = dict(rho_d=np.full(mesh.nzq, rd.mean()), rho_m=np.full(mesh.nzq, rm.mean()),
              rho_r=np.zeros(mesh.nzq), E=np.full(mesh.nzq, E.mean()))
    U = _layout([rd - bg["rho_d"][0], rm - bg["rho_m"][0]] + m + [E - bg["E"][0]])
    umax = float(np.max(np.sqrt(sum(ua * ua for ua in u))))
    dt = cfl_dt(mesh, umax, 0.0, 0.2)
    return Case("periodic-%dd-q%d-%s%s" % (dim, order, "x".join(map(str, n)), _sfx(basis)), mesh, 3 + dim, 0,
                0.0, 0.0, bg, U, dt, nsteps, seed,
                info=dict(T0=T0, sat_fraction_magnus=frac_sat(T0)))


def moist_bubble(n=(128, 64), order=4, seed=2, nsteps=1000, amp=2.0, centre=(10e3, 2e3),
                 radius=2e3, noise=1e-4, ratio=1.3, Ts=300.0, top=10e3, basis="lobatto") -> Case:
    """2D moist rising bubble in a cloudy background (Bryan-Fritsch shape).

    Domain 20 km x `top` (10 km), periodic in x, slip walls in z, gravity on,
    no rain.
    """
    rng = np.random.default_rng(seed)
    mesh = Mesh(2, list(n), [0.0, 0.0], [20e3, top], [PERIODIC, WALL], order, basis)
    bgf = background(mesh, Ts, lambda z: ratio + 0.0 * z)
    X = node_coords(mesh)
    th = bubble(X, centre, radius, amp)
    U = theta_to_state(mesh, bgf, th, rain=False)
    if noise:
        add_noise(rng, U, mesh, _bg_at_nodes(mesh, bgf), rain=False, level=noise)
    dt = cfl_dt(mesh, 5.0, 0.0, 0.2)
    bg = {k: bgf[k] for k in ("rho_d", "rho_m", "rho_r", "E")}
    return Case("bubble-2d-q%d-%dx%d%s" % (order, n[0], n[1], _sfx(basis)), mesh, 5, 0, C["g"], 0.0, bg, U, dt,
                nsteps, seed, bg_full=bgf)


def warm_rain_3d(n=(64, 64, 32), order=3, seed=3, nsteps=500, nbubbles=8, noise=1e-4,
                 vr=5.0, basis="lobatto") -> Case:
    """3D warm-rain thermals: Kessler on, rain falling at a constant 5 m/s.

    Domain 20 x 20 x 10 km, periodic in x and y, slip walls in z.  The background
    is subsaturated below ~1.5 km and cloudy above; eight +2 K bubbles at random
    positions and a Gaussian rain blob 1 km above each.
    """
    rng = np.random.default_rng(seed)
    mesh = Mesh(3, list(n), [0.0, 0.0, 0.0], [20e3, 20e3, 10e3], [PERIODIC, PERIODIC, WALL], order, basis)
    bgf = background(mesh, 300.0, lambda z: 0.8 + 0.25 * (1.0 + np.tanh((z - 1500.0) / 300.0)))
    X = node_coords(mesh)
    th = np.zeros_like(X[0])
    rr = np.zeros_like(X[0])
    for _ in range(nbubbles):
        cx, cy = rng.uniform(2e3, 18e3, size=2)
        cz = rng.uniform(1.5e3, 3e3)
        th += bubble(X, (cx, cy, cz), 2e3, 2.0)
        r2 = (X[0] - cx) ** 2 + (X[1] - cy) ** 2 + (X[2] - cz - 1e3) ** 2
        rr += 1e-3 * np.exp(-r2 / 1e6)
    U = theta_to_state(mesh, bgf, th, rain=True)
    U[2] += rr
    if noise:
        add_noise(rng, U, mesh, _bg_at_nodes(mesh, bgf), rain=True, level=noise)
    dt = cfl_dt(mesh, 5.0, vr, 0.2)
    bg = {k: bgf[k] for k in ("rho_d", "rho_m", "rho_r", "E")}
    return Case("rain-3d-q%d-%dx%dx%d%s" % (order, *n, _sfx(basis)), mesh, 7, 1, C["g"], vr, bg, U, dt, nsteps, seed,
                bg_full=bgf)


def ensemble(nmembers=64, order=3, seed=4, nsteps=200, lo=16, hi=80) -> List[Case]:
    """Uneven ensemble of 2D bubbles: nx = 2*U{lo..hi}, nz = nx/2 per member."""
    rng = np.random.default_rng(seed)
    out = []
    for mbr in range(nmembers):
        nx = 2 * int(rng.integers(lo, hi + 1))
        amp = float(rng.uniform(1.0, 3.0))
        xc = float(rng.uniform(5e3, 15e3))
        zc = float(rng.uniform(1.5e3, 3e3))
        c = moist_bubble(n=(nx, nx // 2), order=order, seed=seed * 1000 + mbr, nsteps=nsteps,
                         amp=amp, centre=(xc, zc))
        c.name = "member%02d-" % mbr + c.name
        out.append(c)
    return out


def _theta_e(T, p, qw):
    """Wet equivalent potential temperature of saturated air at (T, p) with total
    water ratio q_w = rho_m / rho_d (the definition the paper takes from Emanuel)."""
    rvs = paper_rho_vs(T) if qw > 0 else 0.0 * T          # q_w = 0: dry air, theta_e = theta
    rd = (p - rvs * C["Rv"] * T) / (C["Rd"] * T)
    cp = C["cpd"] + C["cl"] * qw
    return T * (rd * C["Rd"] * T / C["pref"]) ** (-C["Rd"] / cp) * \
        np.exp((C["Lref"] + (C["cpv"] - C["cl"]) * (T - C["Tref"])) * rvs / (rd * cp * T))


def _T_of_theta_e(th, p, qw, lo=180.0, hi=340.0, iters=80):
    """Saturated temperature with theta_e(T, p) = th (vectorised bisection; theta_e
    increases with T at fixed p)."""
    th, p = np.broadcast_arrays(np.asarray(th, dtype=np.float64), np.asarray(p, dtype=np.float64))
    a, b = np.full(th.shape, lo), np.full(th.shape, hi)
    for _ in range(iters):
        m = 0.5 * (a + b)
        up = _theta_e(m, p, qw) < th
        a, b = np.where(up, m, a), np.where(up, b, m)
    return 0.5 * (a + b)


def gravity_waves(n=(300, 10), order=3, t_end=3600.0, dtheta=0.01, u0=20.0, qw=0.02, N2=1.0e-4,
                  theta0=300.0, a=5.0e3, cfl=0.5, length=300.0e3, height=10.0e3, periodic=True,
                  basis="lobatto") -> Case:
    """Inertia gravity waves in a saturated atmosphere (Section 4.1; set-up of
    Appendix B.1).

    Domain 300 km x 10 km, periodic in x, slip walls in z, no rain, wind
    u = (20, 0) m/s.
    - Base state: saturated everywhere with total water q_w = rho_m / rho_d =
      0.02, wet equivalent potential temperature theta_e = theta0 exp(N^2 z/g)
      and hydrostatic balance dp/dz = -(1 + q_w) rho_d g from p(0) = p_ref.
    - Perturbation: theta_e' = dtheta sin(pi z/H) / (1 + ((x - L/2)/a)^2) at the
      base-state pressure, with the same q_w, still saturated.  On the periodic
      domain the x-profile has a slope jump at x = 0 = L (about 1e-3 of its
      peak), which caps L2 convergence near h^1.5.  With `periodic` the profile
      is the sum over its periodic images, in closed form
      (pi a / L) sinh(b) / (cosh(b) - cos(2 pi (x - L/2) / L)), b = 2 pi a / L,
      smooth across the boundary and within 2e-3 of the original.
    The construction uses the paper's saturation law (see paper_rho_vs).
    """
    from scipy.integrate import solve_ivp
    g = C["g"]
    mesh = Mesh(2, list(n), [0.0, 0.0], [length, height], [PERIODIC, WALL], order, basis)
    z = node_heights(mesh)

    def the(zz):
        return theta0 * np.exp(N2 * np.asarray(zz) / g)

    def rd_of(zz, p):
        T = _T_of_theta_e(the(zz), p, qw)
        return (p - (paper_rho_vs(T) if qw > 0 else 0.0) * C["Rv"] * T) / (C["Rd"] * T)

    zs = np.unique(np.concatenate([[0.0], z]))
    sol = solve_ivp(lambda zz, p: -(1.0 + qw) * rd_of(zz, p) * g, (0.0, float(zs[-1])), [C["pref"]],
                    t_eval=zs, rtol=1e-12, atol=1e-8, method="DOP853")
    p = np.interp(z, sol.t, sol.y[0])
    T = _T_of_theta_e(the(z), p, qw)
    rvs = paper_rho_vs(T) if qw > 0 else 0.0 * T
    rd = (p - rvs * C["Rv"] * T) / (C["Rd"] * T)
    rm = qw * rd
    E = energy(rd, rvs, rm - rvs, 0.0, T)
    bgf = dict(rho_d=rd, rho_m=rm, rho_r=np.zeros_like(z), E=E, T=T, p=p)
    # perturbed state at the nodes
    X = node_coords(mesh)
    b = _bg_at_nodes(mesh, bgf)
    if periodic:
        bb = 2.0 * np.pi * a / length
        prof = (np.pi * a / length) * np.sinh(bb) / (np.cosh(bb) - np.cos(2.0 * np.pi * (X[0] - 0.5 * length) / length))
    else:
        prof = 1.0 / (1.0 + ((X[0] - 0.5 * length) / a) ** 2)
    thp = dtheta * np.sin(np.pi * X[1] / height) * prof
    Tn = _T_of_theta_e(the(X[1]) + thp, b["p"], qw)
    rvn = paper_rho_vs(Tn) if qw > 0 else 0.0 * Tn
    rdn = (b["p"] - rvn * C["Rv"] * Tn) / (C["Rd"] * Tn)
    rmn = qw * rdn
    rho = rdn + rmn
    En = energy(rdn, rvn, rmn - rvn, 0.0, Tn, rho * u0 * u0)
    U = _layout([rdn - b["rho_d"], rmn - b["rho_m"], rho * u0, np.zeros_like(rho), En - b["E"]])
    dt = cfl_dt(mesh, u0, 0.0, cfl)
    nsteps = int(np.ceil(t_end / dt))
    bg = {k: bgf[k] for k in ("rho_d", "rho_m", "rho_r", "E")}
    return Case("gravity-waves-q%d-%dx%d%s" % (order, *n, _sfx(basis)), mesh, 5, 0, g, 0.0, bg, U, t_end / nsteps, nsteps, 0,
                info=dict(t_end=t_end, qw=qw, N2=N2, u0=u0), bg_full=bgf)


def adjoint_case(n=(64, 32), order=3, seed=5, nsteps=200) -> Case:
    """The bubble used for gradients: dt fixed by the unperturbed set-up."""
    return moist_bubble(n=n, order=order, seed=seed, nsteps=nsteps)


def directions(mesh: Mesh, ndir=16, seed=6, centre=(10e3, 2e3)) -> np.ndarray:
    """Seeded unit directions: sums of four 1 km Gaussian bumps near the bubble."""
    rng = np.random.default_rng(seed)
    X = node_coords(mesh)
    out = []
    for _ in range(ndir):
        f = np.zeros_like(X[0])
        for _ in range(4):
            cx = centre[0] + rng.uniform(-2e3, 2e3)
            cz = centre[1] + rng.uniform(-1e3, 2e3)
            f += rng.standard_normal() * np.exp(-((X[0] - cx) ** 2 + (X[1] - cz) ** 2) / 1e6)
        out.append(f / np.sqrt(np.sum(f * f)))
    return np.stack(out)


# ----------------------------------------------------------------------------
# triangulations (the simplicial meshes of Section 3.1)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class TriMesh:
    """Conforming triangulation of a box in the (x, z) plane.

    Every cell of an n[0] x n[1] grid is cut along its rising diagonal into two
    triangles.  ``xy[e, v]`` holds the counter-clockwise vertices of element e,
    face f joins vertex f and vertex (f + 1) mod 3, ``nb[e, f]`` is the element
    across face f (-1: slip wall) and ``nbf[e, f]`` that element's face; the
    periodic pairs are in the tables.  Element 2 (j n[0] + i) + t is triangle t
    of cell (i, j).  The background is described on the n[1] grid rows.
    """
    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc: Sequence[int]
    order: int
    xy: np.ndarray
    nb: np.ndarray
    nbf: np.ndarray

    @property
    def ne(self) -> int:
        return int(self.xy.shape[0])

    @property
    def npe(self) -> int:
        """Modes per element: the dimension of P^k in two variables."""
        return (self.order + 1) * (self.order + 2) // 2

    @property
    def h(self) -> np.ndarray:
        return (np.asarray(self.hi, float) - np.asarray(self.lo, float)) / np.asarray(self.n, float)

    @property
    def layers(self) -> Mesh:
        """The grid rows as a box mesh: the background lives at its Gauss heights."""
        return Mesh(2, list(self.n), list(self.lo), list(self.hi), list(self.bc), self.order, "gauss")

    @property
    def nzq(self) -> int:
        return self.n[1] * (self.order + 1)


def tri_mesh(n=(8, 4), lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(PERIODIC, WALL), order=2, jitter=0.0,
             seed=0) -> TriMesh:
    """Structured triangulation with optional seeded vertex jitter.

    ``jitter`` moves every vertex by up to that fraction of the cell size per
    axis (uniform random); vertices on a slip wall move only along it, and
    periodic images move together.
    """
    nx, nz = int(n[0]), int(n[1])
    hx, hz = (hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / nz
    rng = np.random.default_rng(seed)
    dxy = jitter * rng.uniform(-1.0, 1.0, size=(nx + 1, nz + 1, 2)) * np.array([hx, hz])
    if bc[0] == PERIODIC:
        dxy[nx] = dxy[0]
    else:
        dxy[0, :, 0] = dxy[nx, :, 0] = 0.0
    if bc[1] == PERIODIC:
        dxy[:, nz] = dxy[:, 0]
    else:
        dxy[:, 0, 1] = dxy[:, nz, 1] = 0.0
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(nz + 1), indexing="ij")
    P = np.stack([lo[0] + I * hx, lo[1] + J * hz], axis=-1) + dxy        # (nx+1, nz+1, 2)
    ne = 2 * nx * nz
    xy = np.zeros((ne, 3, 2))
    nb = np.full((ne, 3), -1, dtype=np.int32)
    nbf = np.full((ne, 3), -1, dtype=np.int32)

    def cell(i, j):
        """First element of cell (i, j) after periodic wrapping, or -1 past a wall."""
        if bc[0] == PERIODIC:
            i %= nx
        if bc[1] == PERIODIC:
            j %= nz
        if not (0 <= i < nx and 0 <= j < nz):
            return -1
        return 2 * (j * nx + i)

    for j in range(nz):
        for i in range(nx):
            e = cell(i, j)
            v00, v10, v11, v01 = P[i, j], P[i + 1, j], P[i + 1, j + 1], P[i, j + 1]
            xy[e] = (v00, v10, v11)
            xy[e + 1] = (v00, v11, v01)
            # lower triangle: bottom edge, right edge, diagonal
            for f, (c2, t2, f2) in enumerate([(cell(i, j - 1), 1, 1), (cell(i + 1, j), 1, 2), (e, 1, 0)]):
                if c2 >= 0:
                    nb[e, f], nbf[e, f] = c2 + t2, f2
            # upper triangle: diagonal, top edge, left edge
            for f, (c2, t2, f2) in enumerate([(e, 0, 2), (cell(i, j + 1), 0, 0), (cell(i - 1, j), 0, 1)]):
                if c2 >= 0:
                    nb[e + 1, f], nbf[e + 1, f] = c2 + t2, f2
    return TriMesh([nx, nz], list(lo), list(hi), list(bc), order, xy, nb, nbf)


@dataclasses.dataclass
class TriCase:
    """A workload on a triangulation: the state is a function of position.

    ``point_state(xz)`` maps coordinates of shape (..., 2) to the perturbation
    state (nvars, ...) there; each solver samples it at its own quadrature
    points and projects onto its basis.  ``bg`` holds rho_d, rho_m, rho_r, E at
    the Gauss heights of the grid rows (``mesh.layers``).
    """
    name: str
    mesh: TriMesh
    nvars: int
    rain: int
    g: float
    vr_const: float
    bg: Dict[str, np.ndarray]
    point_state: Callable[[np.ndarray], np.ndarray]
    dt: float
    nsteps: int
    seed: int


def tri_bubble(n=(64, 32), order=3, seed=7, nsteps=100, amp=2.0, centre=(10e3, 2e3), radius=2e3,
               ratio=1.3, Ts=300.0, top=10e3, jitter=0.0, rain=False, vr=5.0, noise=0.0) -> TriCase:
    """The 2D moist rising bubble of ``moist_bubble`` on a triangulation.

    Domain 20 km x `top`, periodic in x, slip walls in z, gravity on (the
    shape of the paper's bubble run on triangles, Section 4.2).  With ``rain``
    a Gaussian rain blob of 1e-3 kg/m^3 sits 1 km above the bubble and falls at
    ``vr``; ``noise`` adds seeded relative noise of that level at the sample
    points (the same draw for the same array of points).
    """
    mesh = tri_mesh(n, (0.0, 0.0), (20e3, top), (PERIODIC, WALL), order, jitter, seed)
    bgf = background(mesh.layers, Ts, lambda z: ratio + 0.0 * z)
    bg = {k: bgf[k] for k in ("rho_d", "rho_m", "rho_r", "E")}

    def point_state(xz):
        xz = np.asarray(xz, dtype=np.float64)
        X = [xz[..., 0], xz[..., 1]]
        b = background_at(X[1], Ts, lambda z: ratio + 0.0 * z)
        th = bubble(X, centre, radius, amp)
        Tp = th * (b["p"] / C["pref"]) ** (C["Rd"] / C["cpd"])
        E1 = partitioned_energy(b["rho_d"], b["rho_m"], b["rho_r"], b["T"] + Tp)
        E0 = partitioned_energy(b["rho_d"], b["rho_m"], b["rho_r"], b["T"])
        z = np.zeros_like(th)
        flds = [z, z.copy()]
        if rain:
            r2 = (X[0] - centre[0]) ** 2 + (X[1] - centre[1] - 1e3) ** 2
            flds.append(1e-3 * np.exp(-r2 / 1e6))
        flds += [z.copy(), z.copy(), E1 - E0]
        if noise:
            rng = np.random.default_rng(seed)
            rho = b["rho_d"] + b["rho_m"]
            scales = [b["rho_d"], b["rho_m"]] + ([1e-3 + 0.0 * rho] if rain else []) + [rho, rho, b["E"]]
            for v, sc in enumerate(scales):
                flds[v] = flds[v] + noise * sc * rng.standard_normal(th.shape)
        return np.ascontiguousarray(np.stack(flds))

    h = float(np.min(mesh.h))
    dt = float(0.2 * 0.5 * h / ((2 * order + 1) * (C_BOUND + 5.0 + (vr if rain else 0.0))))
    return TriCase("%s-2d-p%d-%dx%dx2%s" % ("rain" if rain else "bubble", order, n[0], n[1],
                                            "-jitter" if jitter else ""), mesh, 6 if rain else 5, int(rain),
                   C["g"], vr if rain else 0.0, bg, point_state, dt, nsteps, seed)
